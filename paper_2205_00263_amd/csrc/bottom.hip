// Fused bottom of a back-substitution pass for networks whose first layer is a
// small convolution of the input followed by a ReLU (ConvSmall, ResNet stems).
//
// One workgroup owns one instance (subproblem, parameter set) and walks its
// rows.  Per row, everything below the first ReLU's output stays on chip:
//   fold of ReLU layer 0 (Eq. 5)                -> ahat in LDS, a' in registers
//   transposed first convolution (Eq. 2)        -> a^(0) in registers
//   concretisation over the box (Eq. 6), x*     -> lb, x* in LDS
//   adjoint: first convolution of x* + bias, the relaxation of ReLU layer 0
//   and the alpha/beta gradient sums of the instance (fixed row order).
// Rows of an intermediate-bound pass whose objective is ReLU layer 1 are built
// directly from the objective convolution's filter (the rows +-e_j).
#include "bottom.h"
#include "../../include/mnbab.h"

#include <stdlib.h>

namespace mnb {

constexpr int BT = 512;     // threads (8 wavefronts)
constexpr int NWV = BT / 64;
constexpr int NJ_MAX = 8;   // owned neurons of ReLU layer 0 per thread (d1 <= 4096)
constexpr int NO = 6;       // input elements per thread (d0 <= 3072)

// Exact n / d for 0 <= n < 2^22 and 0 < d via a float reciprocal and one correction.
struct FastDiv {
    int d;
    float inv;
    __device__ FastDiv(int d_) : d(d_), inv(1.0f / (float)d_) {}
    __device__ __forceinline__ int div(int n) const {
        int q = (int)((float)n * inv);
        if ((q + 1) * d <= n) ++q;
        if (q * d > n) --q;
        return q;
    }
};

// Workgroup barrier that orders LDS accesses only: outstanding global loads (the next
// row's prefetch) stay in flight across it.  No global data written in the row loop is
// read back by another thread of the workgroup.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum of three per-thread values over the block (fixed order); one barrier.
__device__ __forceinline__ void block_sum3(float& x, float& y, float& z, float (*red)[NWV]) {
    x = wave_sum(x);
    y = wave_sum(y);
    z = wave_sum(z);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = x;
        red[1][w] = y;
        red[2][w] = z;
    }
    lds_barrier();
    x = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3])) + ((red[0][4] + red[0][5]) + (red[0][6] + red[0][7]));
    y = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3])) + ((red[1][4] + red[1][5]) + (red[1][6] + red[1][7]));
    z = ((red[2][0] + red[2][1]) + (red[2][2] + red[2][3])) + ((red[2][4] + red[2][5]) + (red[2][6] + red[2][7]));
}

// KS: kernel size and stride of the first convolution as compile-time constants
// (0: taken from the arguments).
typedef float floatx4 __attribute__((ext_vector_type(4)));

// MF: the two first-layer convolutions run on v_mfma_f32_16x16x4_f32 (needs CO == 16 and
// Ci*k*k <= 32): the transposed one as T = ahat^T W (positions x taps) plus a col2im
// gather, the adjoint one as im2col(x*) W^T (positions x output channels).
template <int NJ, int KK, int SS, int CO, bool MF>
__global__ __launch_bounds__(BT, (NJ <= 6 ? 4 : 2)) void k_bottom(BottomArgs a) {
    extern __shared__ float smem[];
    const int d1 = a.d1;
    const int k = KK ? KK : a.k;
    const int s = SS ? SS : a.s;
    float* s_ah = smem;                 // [d1]  ahat of the current row, then ghat
    float* s_x = s_ah + d1;             // [d0]  x* of the current row
    float* s_b1 = s_x + a.d0;           // [Co]  first-layer bias per channel
    float* s_w = s_b1 + ((a.Co + 3) & ~3);          // [Co*Ci*k*k] first-layer weights
    float* s_wp = s_w + ((a.Co * a.Ci * a.k * a.k + 3) & ~3);  // [16][32] weights, taps zero-padded (MF only)
    float* s_T = s_wp + (MF ? 16 * 32 : 0);                     // [TS][Ho*Wo] tap products, tap-major (MF only)
    const int TS = a.Ci * a.k * a.k > 16 ? 32 : 16;
    float* s_sh = s_T + (MF ? a.Ho * a.Wo * TS : 0);   // [d1] sum over rows of ghat (own j)
    float* s_sg = s_sh + d1;                           // [d1] sum over rows of g (own j, MNC only)
    float* s_lo = s_sg + d1;                           // [d0] input box of the query (box_lds)
    float* s_hi = s_lo + a.d0;                         // [d0]
    __shared__ float red[3][NWV];

    const int ib = a.cinst[blockIdx.x];
    const InstDesc in = a.inst[ib];
    const int t = threadIdx.x;
    const int kk = k * k;
    const int nw = a.Co * a.Ci * kk;
    const int HoWo = a.Ho * a.Wo, HiWi = a.Hi * a.Wi;
    for (int i = t; i < nw; i += BT) s_w[i] = a.W1[i];
    if constexpr (MF)
        for (int i = t; i < 16 * 32; i += BT) {
            const int co = i >> 5, tap = i & 31;
            s_wp[i] = tap < a.Ci * kk ? a.W1[co * a.Ci * kk + tap] : 0.f;
        }
    for (int i = t; i < a.Co; i += BT) s_b1[i] = a.b1[i];
    const float* glo = a.lo + (long)a.qid[in.slot] * a.d0;
    const float* ghi = a.hi + (long)a.qid[in.slot] * a.d0;
    if (a.box_lds)
        for (int o = t; o < a.d0; o += BT) {
            s_lo[o] = glo[o];
            s_hi[o] = ghi[o];
        }
    // relaxation of ReLU layer 0 for this instance (split first, then stable, then unstable),
    // held by the thread that owns each neuron: slope where a' >= 0, slope and intercept where
    // a' < 0 (the intercept is > 0 exactly when unstable), S beta + (Phat^T gamma)
    float rx_dp[NJ], rx_dn[NJ], rx_bn[NJ], rx_ad[NJ];
    unsigned split_bits = 0;   // bit i: neuron t + i BT is split
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const int j = t + i * BT;
        float dp = 0.f, dn = 0.f, bn = 0.f, ad = 0.f;
        if (j < d1) {
            s_sh[j] = 0.f;
            s_sg[j] = 0.f;
            const long so = (long)in.slot * a.ld_state + j;
            const long po = ((long)in.slot * a.n_sets + in.set) * a.ld_param + j;
            const float l = a.l[so], u = a.u[so];
            const int sj = (int)a.S[so];
            if (sj == -1) {
                dp = dn = 1.f;
            } else if (sj == 1) {
            } else if (l >= 0.f) {
                dp = dn = 1.f;
            } else if (u <= 0.f) {
            } else {
                dp = a.alpha[po];
                const float w = u - l;
                dn = u / w;
                bn = -(u * l) / w;
            }
            ad = (sj != 0 ? (float)sj * a.beta[po] : 0.f) + (a.vhat ? a.vhat[(long)ib * d1 + j] : 0.f);
            if (sj != 0) split_bits |= 1u << i;
        }
        rx_dp[i] = dp;
        rx_dn[i] = dn;
        rx_bn[i] = bn;
        rx_ad[i] = ad;
    }
    // forward convolution: per owned neuron its window origin and weight row
    const FastDiv div_HoWo(HoWo), div_Wo(a.Wo), div_HiWi(HiWi), div_Wi(a.Wi);
    const float* vrow = a.v ? a.v + (long)ib * d1 : nullptr;
    float da[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) da[i] = 0.f;
    const bool want_h = a.gsum_hat != nullptr;
    const float gpv = a.gp ? a.gp[ib] : 0.f;
    const int q = a.qid[in.slot];

    __syncthreads();
    const int lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
    const int ntap = a.Ci * kk;                  // taps (ci, ky, kx) of one output channel
    const int MT = (HoWo + 15) >> 4;             // 16-row tiles over the positions of ReLU layer 0
    // MFMA B operands are read from s_wp per tile: transposed B[k = co][n = tap],
    // adjoint B[k = tap][n = co]

    for (int r = a.cr0[blockIdx.x]; r < a.cr1[blockIdx.x]; ++r) {
        const RowDesc rd = a.rows[r];
        // previous bound of the row (thread 0): each (slot, neuron) of the objective layer has
        // exactly one row in a pass
        float old = 0.f;
        if (t == 0) {
            if (a.mode == 0) {
                const long e = (long)in.slot * a.ld_state + a.state_off_obj + rd.j;
                old = rd.sign > 0 ? a.lw[e] : a.uw[e];
            } else if (a.mode == 1) {
                old = a.best[r];
            }
        }
        // ---- row coefficients on the output of ReLU layer 0 (each thread its own j)
        float crow = 0.f;
        float ap[NJ];
        if (a.src_mode == 0) {
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                const int j = t + i * BT;
                ap[i] = j < d1 ? a.A[(long)r * d1 + j] : 0.f;
            }
            if (t == 0) {
                crow = a.c[r];
                for (int kq = 0; kq < a.ncp; ++kq) crow += a.cpart[(long)r * a.ldcp + kq];
            }
        } else {
            // +-e_j on the output of the objective convolution: its filter placed at j
            const float sgn = (float)rd.sign;
            const int per = a.oHo * a.oWo;
            const int co = rd.j / per;
            const int pos = rd.j - co * per;
            const int y = pos / a.oWo, x = pos - y * a.oWo;
            const int oHiWi = a.oHi * a.oWi;
            const FastDiv div_o(oHiWi), div_ow(a.oWi);
            const float* wrow = a.Wobj + (long)co * a.oCi * a.ok * a.ok;
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                const int j = t + i * BT;
                float v = 0.f;
                if (j < d1) {
                    const int ci = div_o.div(j);
                    const int qq = j - ci * oHiWi;
                    const int Y = div_ow.div(qq), X = qq - Y * a.oWi;
                    const int ky = Y - a.os * y + a.op, kx = X - a.os * x + a.op;
                    if ((unsigned)ky < (unsigned)a.ok && (unsigned)kx < (unsigned)a.ok)
                        v = sgn * wrow[(ci * a.ok + ky) * a.ok + kx];
                }
                ap[i] = v;
            }
            if (t == 0) crow = sgn * a.bias_obj[rd.j];
        }
        // ---- fold of ReLU layer 0
        float cpt = 0.f;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const int j = t + i * BT;
            if (j < d1) {
                const float p = ap[i] + (vrow ? vrow[j] : 0.f);
                ap[i] = p;
                const bool neg = p < 0.f;
                const float ah = p * (neg ? rx_dn[i] : rx_dp[i]) + rx_ad[i];
                s_ah[j] = ah;
                cpt += (neg ? p * rx_bn[i] : 0.f) + ah * s_b1[div_HoWo.div(j)];
                if (a.Ap_out) a.Ap_out[(long)r * d1 + j] = p;
            }
        }
        if (t == 0) cpt += crow - gpv;
        lds_barrier();
        // ---- transposed first convolution and concretisation
        float lbp = 0.f, mag = 0.f;
        const int wst = a.Ci * kk;
        if constexpr (MF) {
            // T[pos][tap] = sum_co ahat[co][pos] W[co][tap]
            const int NTT = ntap > 16 ? 2 : 1;
            for (int mt = wave; mt < MT; mt += NWV) {
                const int pos = mt * 16 + lr;
                float av[4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) av[ks] = pos < HoWo ? s_ah[(ks * 4 + lk) * HoWo + pos] : 0.f;
                for (int nt = 0; nt < NTT; ++nt) {
                    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks], s_wp[(ks * 4 + lk) * 32 + nt * 16 + lr], acc, 0, 0, 0);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int p2 = mt * 16 + 4 * lk + v;
                        if (p2 < HoWo) s_T[(nt * 16 + lr) * HoWo + p2] = acc[v];   // tap-major
                    }
                }
            }
            lds_barrier();
        }
        for (int o = t; o < a.d0; o += BT) {
            const int ci = div_HiWi.div(o);
            const int qq = o - ci * HiWi;
            const int Yq = div_Wi.div(qq);
            const int Yp = Yq + a.p, Xp = qq - Yq * a.Wi + a.p;
            float acc = 0.f;
#pragma unroll
            for (int ty = 0; ty < (KK ? (KK + SS - 1) / SS : 8); ++ty) {
                const int ky = Yp % s + ty * s;
                if (!KK && ky >= k) break;
                const int y = (Yp - ky) / s;
                if (ky >= k || y < 0 || y >= a.Ho) continue;
#pragma unroll
                for (int tx = 0; tx < (KK ? (KK + SS - 1) / SS : 8); ++tx) {
                    const int kx = Xp % s + tx * s;
                    if (!KK && kx >= k) break;
                    const int x = (Xp - kx) / s;
                    if (kx >= k || x < 0 || x >= a.Wo) continue;
                    if constexpr (MF) {
                        acc += s_T[((ci * k + ky) * k + kx) * HoWo + y * a.Wo + x];
                        continue;
                    }
                    const float* ah = s_ah + y * a.Wo + x;
                    const float* w = s_w + (ci * k + ky) * k + kx;
                    if (CO) {
                        float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int co = 0; co < (CO ? CO : 1); ++co) part[co & 3] += ah[co * HoWo] * w[co * wst];
                        acc += (part[0] + part[1]) + (part[2] + part[3]);
                    } else {
                        for (int co = 0; co < a.Co; ++co) acc += ah[co * HoWo] * w[co * wst];
                    }
                }
            }
            float l, h;
            if (a.box_lds) {
                l = s_lo[o];
                h = s_hi[o];
            } else {
                l = glo[o];
                h = ghi[o];
            }
            lbp += fminf(acc * l, acc * h);
            mag += fabsf(acc) * fmaxf(fabsf(l), fabsf(h));
            const bool neg = acc < 0.f;
            s_x[o] = neg ? h : l;
            if (a.xbits) a.xbits[(long)r * a.d0 + o] = neg ? 1 : 0;
        }
        block_sum3(lbp, mag, cpt, red);   // also publishes s_x
        if (t == 0) {
            float lb = (lbp + cpt) - (mag + fabsf(cpt)) * 9.5367431640625e-07f;   // 2^-20 rounding margin
            if (!(lb == lb) || isinf(lb)) lb = -INFINITY;
            if (a.mode == 0) {
                // each (slot, neuron) of the objective layer has exactly one row in a pass
                const long e = (long)in.slot * a.ld_state + a.state_off_obj + rd.j;
                if (rd.sign > 0)
                    a.lw[e] = fmaxf(old, lb);
                else
                    a.uw[e] = fminf(old, isinf(lb) ? INFINITY : -lb);
            } else {
                a.lb_out[r] = lb;
                if (a.mode == 1) {
                    const bool better = lb > old;
                    if (better) a.best[r] = lb;
                    a.improved[r] = better ? 1 : 0;
                }
            }
        }
        if (a.adjoint) {
            // ---- adjoint: first convolution of x* into s_ah (ahat is no longer read) ...
            if constexpr (MF) {
                const int KS = (ntap + 3) >> 2;
                for (int mt = wave; mt < MT; mt += NWV) {
                    const int pos = mt * 16 + lr;
                    const int y = div_Wo.div(pos), x = pos - y * a.Wo;
                    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 8; ++ks) {
                        if (ks >= KS) break;
                        const int kq = ks * 4 + lk;
                        float av = 0.f;
                        if (kq < ntap && pos < HoWo) {
                            const int ci = kq / kk, rr = kq - ci * kk;
                            const int ky = rr / k, kx = rr - ky * k;
                            const int Y = s * y - a.p + ky, X = s * x - a.p + kx;
                            if ((unsigned)Y < (unsigned)a.Hi && (unsigned)X < (unsigned)a.Wi)
                                av = s_x[(ci * a.Hi + Y) * a.Wi + X];
                        }
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, s_wp[lr * 32 + ks * 4 + lk], acc, 0, 0, 0);
                    }
                    const float bco = a.b1[lr];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int p2 = mt * 16 + 4 * lk + v;
                        if (p2 < HoWo) s_ah[lr * HoWo + p2] = acc[v] + bco;
                    }
                }
                lds_barrier();
            } else
            for (int j = t; j < d1; j += BT) {
                const int co = div_HoWo.div(j);
                const int qq = j - co * HoWo;
                const int y = div_Wo.div(qq), x = qq - y * a.Wo;
                const int Y0 = s * y - a.p, X0 = s * x - a.p;
                const float* w = s_w + co * a.Ci * kk;
                float gh = a.b1[co];
                if (Y0 >= 0 && X0 >= 0 && Y0 + k <= a.Hi && X0 + k <= a.Wi) {
                    const float* xp = s_x + Y0 * a.Wi + X0;
                    for (int ci = 0; ci < a.Ci; ++ci) {
                        if (KK) {
#pragma unroll
                            for (int ky = 0; ky < (KK ? KK : 1); ++ky)
#pragma unroll
                                for (int kx = 0; kx < (KK ? KK : 1); ++kx)
                                    gh += w[(ci * KK + ky) * KK + kx] * xp[ci * HiWi + ky * a.Wi + kx];
                        } else {
                            for (int ky = 0; ky < k; ++ky)
                                for (int kx = 0; kx < k; ++kx)
                                    gh += w[(ci * k + ky) * k + kx] * xp[ci * HiWi + ky * a.Wi + kx];
                        }
                    }
                } else {
                    for (int ci = 0; ci < a.Ci; ++ci)
                        for (int ky = 0; ky < k; ++ky) {
                            const int Y = Y0 + ky;
                            if ((unsigned)Y >= (unsigned)a.Hi) continue;
                            for (int kx = 0; kx < k; ++kx) {
                                const int X = X0 + kx;
                                if ((unsigned)X >= (unsigned)a.Wi) continue;
                                gh += w[(ci * k + ky) * k + kx] * s_x[ci * HiWi + Y * a.Wi + X];
                            }
                        }
                }
                s_ah[j] = gh;
            }
            // ... then the relaxation of ReLU layer 0 and the instance's gradient sums (own j only)
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                const int j = t + i * BT;
                if (j < d1) {
                    const float gh = s_ah[j];
                    const bool neg = ap[i] < 0.f;
                    const float bn = rx_bn[i];
                    const float g = (neg ? rx_dn[i] : rx_dp[i]) * gh + (neg ? bn : 0.f);
                    if (bn > 0.f && !neg) da[i] += ap[i] * gh;
                    if (want_h || ((split_bits >> i) & 1u)) s_sh[j] += gh;
                    if (a.gsum_out) s_sg[j] += g;
                    if (a.Gout) a.Gout[(long)r * d1 + j] = g;
                }
            }
        }
        lds_barrier();   // red[] and s_x are rewritten by the next row
    }
    if (!a.adjoint) return;
    // partial sums of this chunk: alpha only where the neuron is unstable, the ghat sum only
    // where it is split or MNC sums are wanted, the g sum only for MNCs (the reduction reads
    // exactly the same entries)
    float* pt = a.part + (long)blockIdx.x * 3 * d1;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const int j = t + i * BT;
        if (j < d1) {
            if (rx_bn[i] > 0.f) pt[j] = da[i];
            if (want_h || ((split_bits >> i) & 1u)) pt[d1 + j] = s_sh[j];
            if (a.gsum_out) pt[2 * d1 + j] = s_sg[j];
        }
    }
}

// Instance gradients: the chunk partials summed in chunk order.
__global__ void k_bottom_reduce(BottomArgs a) {
    const int ib = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= a.d1) return;
    const InstDesc in = a.inst[ib];
    const long so = (long)in.slot * a.ld_state + j;
    const int sj = (int)a.S[so];
    // unstable exactly where the fold used the triangle (same test as the kernel)
    const float l = a.l[so], u = a.u[so];
    const bool unst = sj == 0 && !(l >= 0.f) && !(u <= 0.f) && (-(u * l) / (u - l)) > 0.f;
    const bool need_h = a.gsum_hat || sj != 0;
    float da = 0.f, sh = 0.f, sg = 0.f;
    for (int c = a.ichunk0[ib]; c < a.ichunk1[ib]; ++c) {
        const float* pt = a.part + (long)c * 3 * a.d1;
        if (unst) da += pt[j];
        if (need_h) sh += pt[a.d1 + j];
        if (a.gsum_out) sg += pt[2 * a.d1 + j];
    }
    const long go = (long)ib * a.ldg + j;
    a.d_alpha[go] = da;
    a.d_beta[go] = (float)sj * sh;
    if (a.gsum_hat) a.gsum_hat[(long)ib * a.d1 + j] = sh;
    if (a.gsum_out) a.gsum_out[(long)ib * a.d1 + j] = sg;
}

bool bottom_supported(int d1, int d0, int n_weights) {
    return d1 <= NJ_MAX * BT && d0 <= NO * BT && n_weights <= 4096 &&
           (3 * d1 + d0 + n_weights + 64) * sizeof(float) <= 150 * 1024;
}

template <int KK, int SS, int CO, bool MF>
static void launch_bottom_k(const BottomArgs& a, int n_blk, size_t lds, hipStream_t st) {
    const int nj = cdiv(a.d1, BT);
    if (nj <= 2)
        hipLaunchKernelGGL((k_bottom<2, KK, SS, CO, MF>), dim3(n_blk), dim3(BT), lds, st, a);
    else if (nj <= 4)
        hipLaunchKernelGGL((k_bottom<4, KK, SS, CO, MF>), dim3(n_blk), dim3(BT), lds, st, a);
    else if (nj <= 6)
        hipLaunchKernelGGL((k_bottom<6, KK, SS, CO, MF>), dim3(n_blk), dim3(BT), lds, st, a);
    else
        hipLaunchKernelGGL((k_bottom<8, KK, SS, CO, MF>), dim3(n_blk), dim3(BT), lds, st, a);
}

void launch_bottom(const BottomArgs& a, int n_inst, hipStream_t st) {
    if (n_inst <= 0) return;
    MNB_CHECK(bottom_supported(a.d1, a.d0, a.Co * a.Ci * a.k * a.k) && a.k <= 3 * a.s && (a.s >= 2 || a.k <= 3),
              MNB_EDEVICE, "bottom kernel: unsupported shape");
    const size_t base = (size_t)(3 * a.d1 + a.d0 + ((a.Co + 3) & ~3) + ((a.Co * a.Ci * a.k * a.k + 3) & ~3));
    const size_t ts = a.Ci * a.k * a.k > 16 ? 32 : 16;
    const int nb = a.n_chunk;
    if (nb <= 0) return;
    const bool mf = a.Co == 16 && a.Ci * a.k * a.k <= 32 &&
                    (base + (size_t)a.Ho * a.Wo * ts + 16 * 32) * sizeof(float) <= 150 * 1024 && !getenv("MNB_BOTTOM_VALU");
    size_t lds = (base + (mf ? (size_t)a.Ho * a.Wo * ts + 16 * 32 : 0)) * sizeof(float);
    // the query's box in LDS when it fits beside the rest
    BottomArgs b = a;
    b.box_lds = lds + 2 * (size_t)a.d0 * sizeof(float) <= 150 * 1024;
    if (b.box_lds) lds += 2 * (size_t)a.d0 * sizeof(float);
    if (mf && a.k == 4 && a.s == 2)
        launch_bottom_k<4, 2, 16, true>(b, nb, lds, st);
    else if (mf && a.k == 3 && a.s == 2)
        launch_bottom_k<3, 2, 16, true>(b, nb, lds, st);
    else if (mf)
        launch_bottom_k<0, 0, 16, true>(b, nb, lds, st);
    else if (a.k == 4 && a.s == 2 && a.Co == 16)
        launch_bottom_k<4, 2, 16, false>(b, nb, lds, st);
    else if (a.k == 3 && a.s == 2 && a.Co == 16)
        launch_bottom_k<3, 2, 16, false>(b, nb, lds, st);
    else
        launch_bottom_k<0, 0, 0, false>(b, nb, lds, st);
    MNB_HIP(hipGetLastError());
}

void launch_bottom_reduce(const BottomArgs& a, int n_inst, hipStream_t st) {
    if (!a.adjoint || n_inst <= 0 || a.n_chunk <= 0) return;
    hipLaunchKernelGGL(k_bottom_reduce, dim3(cdiv(a.d1, 256), n_inst), dim3(256), 0, st, a);
    MNB_HIP(hipGetLastError());
}

}  // namespace mnb
