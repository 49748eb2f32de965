// Fused bottom of a back-substitution pass for networks whose first layer is a
// small convolution of the input followed by a ReLU (generic shapes; convolutions
// into 16 channels with at most 32 taps per channel use the MFMA kernel of
// bottom_mf.hip instead).
//
// One workgroup owns one chunk of rows of one instance (subproblem, parameter set)
// and walks its rows.  Per row, everything below the first ReLU's output stays on chip:
//   fold of ReLU layer 0 (Eq. 5)                -> ahat in LDS, a' in registers
//   transposed first convolution (Eq. 2)        -> a^(0) in registers
//   concretisation over the box (Eq. 6), x*     -> lb, x* in LDS
//   adjoint: first convolution of x* + bias, the relaxation of ReLU layer 0
//   and the alpha gradient sums of the instance (fixed row order).
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

// Generic shapes (any first-layer channel count and kernel); the first-layer convolutions
// into 16 channels with at most 32 taps run on MFMA in bottom_mf.hip.
// SRC1: rows built from the objective convolution's filter (src_mode 1), a separate
// instantiation so that the common case carries none of its registers.
// RXL (up to 6 owned neurons per thread): the instance's relaxation of ReLU layer 0 lives
// in LDS as one float4 per neuron instead of in registers, which leaves the registers for
// the next row's prefetched coefficients.
template <int NJ, bool SRC1>
__global__ __launch_bounds__(BT, (NJ <= 6 ? 4 : 2)) void k_bottom(BottomArgs a) {
    constexpr bool RXL = NJ <= 6;
    extern __shared__ float4 smem4[];
    float4* s_rx = smem4;               // [d1] (RXL) {slope a' >= 0, slope a' < 0, intercept, S beta + Phat^T gamma}
    float* smem = reinterpret_cast<float*>(smem4) + (RXL ? 4 * a.d1 : 0);
    const int d1 = a.d1;
    const int k = a.k;
    const int s = a.s;
    float* s_ah = smem;                 // [d1]  ahat of the current row, then ghat
    float* s_x = s_ah + d1;             // [d0]  x* of the current row
    int* s_xc = reinterpret_cast<int*>(s_x + a.d0);   // [d0] rows of the chunk with x*_o = hi_o (own o)
    float* s_b1 = s_x + 2 * a.d0;       // [Co]  first-layer bias per channel
    float* s_w = s_b1 + ((a.Co + 3) & ~3);          // [Co*Ci*k*k] first-layer weights
    float* s_sg = s_w + ((a.Co * a.Ci * a.k * a.k + 3) & ~3);   // [d1] sum of g (own j, MNC only)
    float* s_lo = s_sg + (a.gsum_out ? d1 : 0);        // [d0] input box of the query (box_lds)
    float* s_hi = s_lo + a.d0;                         // [d0]
    __shared__ float red[3][NWV];
    __shared__ RowDesc s_rd[BOTTOM_CHUNK_ROWS];   // the chunk's row descriptors,
    __shared__ float s_crow[BOTTOM_CHUNK_ROWS];   // row constants
    __shared__ float s_old[BOTTOM_CHUNK_ROWS];    // and previous bounds

    const int ib = a.cinst[blockIdx.x];
    const InstDesc in = a.inst[ib];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    // the chunk's rows (at most BOTTOM_CHUNK_ROWS by construction of the chunks): descriptor,
    // constant and previous bound of each, loaded once with all loads in flight together
    const int cr0 = a.cr0[blockIdx.x];
    const int nr = min(a.cr1[blockIdx.x] - cr0, BOTTOM_CHUNK_ROWS);
    for (int ri = wave; ri < nr; ri += NWV) {
        const int r = cr0 + ri;
        float cr = SRC1 ? 0.f : row_constant(a.c, a.cpart, a.ldcp, a.ncp, r);
        if (lane == 0) {
            const RowDesc rd = a.rows[r];
            if (SRC1) cr = (float)rd.sign * a.bias_obj[rd.j];
            float old = 0.f;
            if (a.mode == 0) {
                // each (slot, neuron) of the objective layer has exactly one row in a pass
                const long e = (long)in.slot * a.ld_state + a.state_off_obj + rd.j;
                old = rd.sign > 0 ? a.lw[e] : a.uw[e];
            } else if (a.mode == 1) {
                old = a.best[r];
            }
            s_rd[ri] = rd;
            s_crow[ri] = cr;
            s_old[ri] = old;
        }
    }
    const int kk = k * k;
    const int nw = a.Co * a.Ci * kk;
    const int HoWo = a.Ho * a.Wo, HiWi = a.Hi * a.Wi;
    for (int i = t; i < nw; i += BT) s_w[i] = a.W1[i];
    for (int i = t; i < a.Co; i += BT) s_b1[i] = a.b1[i];
    for (int o = t; o < a.d0; o += BT) s_xc[o] = 0;
    const float* glo = a.lo + (long)a.qid[in.slot] * a.d0;
    const float* ghi = a.hi + (long)a.qid[in.slot] * a.d0;
    const bool box_lds = RXL || a.box_lds;   // RXL launches always stage the box (checked by the host)
    if (box_lds)
        for (int o = t; o < a.d0; o += BT) {
            s_lo[o] = glo[o];
            s_hi[o] = ghi[o];
        }
    // relaxation of ReLU layer 0 for this instance (split first, then stable, then unstable),
    // held by the thread that owns each neuron: slope where a' >= 0, slope and intercept where
    // a' < 0 (the intercept is > 0 exactly when unstable), S beta + (Phat^T gamma)
    constexpr int NR = RXL ? 1 : NJ;
    float rx_dp[NR], rx_dn[NR], rx_bn[NR], rx_ad[NR];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const int j = t + i * BT;
        float dp = 0.f, dn = 0.f, bn = 0.f, ad = 0.f;
        if (j < d1) {
            if (a.gsum_out) s_sg[j] = 0.f;
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
        }
        if constexpr (RXL) {
            if (j < d1) s_rx[j] = make_float4(dp, dn, bn, ad);
        } else {
            rx_dp[i] = dp;
            rx_dn[i] = dn;
            rx_bn[i] = bn;
            rx_ad[i] = ad;
        }
    }
    // relaxation of owned neuron i: registers, or LDS (RXL)
    auto relax = [&](int i) -> float4 {
        if constexpr (RXL)
            return s_rx[t + i * BT];
        else
            return make_float4(rx_dp[i], rx_dn[i], rx_bn[i], rx_ad[i]);
    };
    // forward convolution: per owned neuron its window origin and weight row
    const FastDiv div_HoWo(HoWo), div_Wo(a.Wo), div_HiWi(HiWi), div_Wi(a.Wi);
    const float* vrow = a.v ? a.v + (long)ib * d1 : nullptr;
    float da[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) da[i] = 0.f;
    const float gpv = a.gp ? a.gp[ib] : 0.f;
    // coefficients of the next row, loaded one row ahead (the first row's before the barrier,
    // which waits for them)
    float nx[SRC1 ? 1 : NJ];
    if constexpr (!SRC1) {
#pragma unroll
        for (int i = 0; i < NJ; ++i) nx[i] = (t + i * BT < d1 && nr > 0) ? a.A[(long)cr0 * d1 + t + i * BT] : 0.f;
    }
    __syncthreads();

    for (int ri = 0; ri < nr; ++ri) {
        const int r = cr0 + ri;
        const RowDesc rd = s_rd[ri];
        // ---- row coefficients on the output of ReLU layer 0 (each thread its own j)
        float ap[NJ];
        if constexpr (!SRC1) {
#pragma unroll
            for (int i = 0; i < NJ; ++i) ap[i] = nx[i];
            if (ri + 1 < nr) {
#pragma unroll
                for (int i = 0; i < NJ; ++i)
                    nx[i] = t + i * BT < d1 ? a.A[(long)(r + 1) * d1 + t + i * BT] : 0.f;
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
        }
        // ---- fold of ReLU layer 0 (global loads and stores kept out of the per-element code,
        // so that no element waits for another's memory operations)
        if (vrow) {
            float vv[NJ];
#pragma unroll
            for (int i = 0; i < NJ; ++i) vv[i] = t + i * BT < d1 ? vrow[t + i * BT] : 0.f;
#pragma unroll
            for (int i = 0; i < NJ; ++i) ap[i] += vv[i];
        }
        float cpt = 0.f;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const int j = t + i * BT;
            if (j < d1) {
                const float p = ap[i];
                const bool neg = p < 0.f;
                const float4 rx = relax(i);
                const float ah = p * (neg ? rx.y : rx.x) + rx.w;
                s_ah[j] = ah;
                cpt += (neg ? p * rx.z : 0.f) + ah * s_b1[div_HoWo.div(j)];
            }
        }
        if (a.Ap_out) {
#pragma unroll
            for (int i = 0; i < NJ; ++i)
                if (t + i * BT < d1) a.Ap_out[(long)r * d1 + t + i * BT] = ap[i];
        }
        if (t == 0) cpt += s_crow[ri] - gpv;
        lds_barrier();
        // ---- transposed first convolution and concretisation
        float lbp = 0.f, mag = 0.f;
        const int wst = a.Ci * kk;
        for (int o = t; o < a.d0; o += BT) {
            const int ci = div_HiWi.div(o);
            const int qq = o - ci * HiWi;
            const int Yq = div_Wi.div(qq);
            const int Yp = Yq + a.p, Xp = qq - Yq * a.Wi + a.p;
            float acc = 0.f;
#pragma unroll
            for (int ty = 0; ty < 8; ++ty) {
                const int ky = Yp % s + ty * s;
                if (ky >= k) break;
                const int y = (Yp - ky) / s;
                if (y < 0 || y >= a.Ho) continue;
#pragma unroll
                for (int tx = 0; tx < 8; ++tx) {
                    const int kx = Xp % s + tx * s;
                    if (kx >= k) break;
                    const int x = (Xp - kx) / s;
                    if (x < 0 || x >= a.Wo) continue;
                    const float* ah = s_ah + y * a.Wo + x;
                    const float* w = s_w + (ci * k + ky) * k + kx;
                    for (int co = 0; co < a.Co; ++co) acc += ah[co * HoWo] * w[co * wst];
                }
            }
            float l, h;
            if (box_lds) {
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
            if (a.adjoint && neg) s_xc[o] += 1;
            if (a.xbits) a.xbits[(long)r * a.d0 + o] = neg ? 1 : 0;
        }
        block_sum3(lbp, mag, cpt, red);   // also publishes s_x
        if (t == 0) {
            float lb = (lbp + cpt) - (mag + fabsf(cpt)) * a.margin;   // rounding margin of spec rows
            if (!(lb == lb) || isinf(lb)) lb = -INFINITY;
            const float old = s_old[ri];
            if (a.mode == 0) {
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
            for (int j = t; j < d1; j += BT) {
                const int co = div_HoWo.div(j);
                const int qq = j - co * HoWo;
                const int y = div_Wo.div(qq), x = qq - y * a.Wo;
                const int Y0 = s * y - a.p, X0 = s * x - a.p;
                const float* w = s_w + co * a.Ci * kk;
                float gh = s_b1[co];
                if (Y0 >= 0 && X0 >= 0 && Y0 + k <= a.Hi && X0 + k <= a.Wi) {
                    const float* xp = s_x + Y0 * a.Wi + X0;
                    for (int ci = 0; ci < a.Ci; ++ci)
                        for (int ky = 0; ky < k; ++ky)
                            for (int kx = 0; kx < k; ++kx)
                                gh += w[(ci * k + ky) * k + kx] * xp[ci * HiWi + ky * a.Wi + kx];
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
            float gv[NJ];
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                const int j = t + i * BT;
                gv[i] = 0.f;
                if (j < d1) {
                    const float gh = s_ah[j];
                    const bool neg = ap[i] < 0.f;
                    const float4 rx = relax(i);
                    const float bn = rx.z;
                    const float g = (neg ? rx.y : rx.x) * gh + (neg ? bn : 0.f);
                    if (bn > 0.f && !neg) da[i] += ap[i] * gh;
                    if (a.gsum_out) s_sg[j] += g;
                    gv[i] = g;
                }
            }
            vmem_drain();
            if (a.Gout) {
#pragma unroll
                for (int i = 0; i < NJ; ++i)
                    if (t + i * BT < d1) a.Gout[(long)r * d1 + t + i * BT] = gv[i];
            }
        } else {
            vmem_drain();
        }
        lds_barrier();   // red[] and s_x are rewritten by the next row
    }
    if (!a.adjoint) return;
    // partial sums of this chunk: alpha only where the neuron is unstable, the g sum only for
    // MNCs (the reduction reads exactly the same entries), and per input element the number
    // of rows with x* = hi, from which the reduction takes the ghat sum (ghat = W1 x* + b1 is
    // affine in x*, and x* is a box corner)
    float* pt = a.part + (long)blockIdx.x * (2 * d1 + a.d0);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const int j = t + i * BT;
        if (j < d1) {
            if (relax(i).z > 0.f) pt[j] = da[i];
            if (a.gsum_out) pt[d1 + j] = s_sg[j];
        }
    }
    for (int o = t; o < a.d0; o += BT) pt[2 * d1 + o] = (float)s_xc[o];
}

// Instance gradients: the chunk partials summed in chunk order.  The sum over the n rows of
// ghat_j is (W1 X)_j + n b1 with X_o = m_o hi_o + (n - m_o) lo_o, m_o the number of rows
// with x*_o = hi_o (exact); it is evaluated in double, free of the cancellation that a
// float sum of nearly opposite row terms would suffer.
// One neuron j of ReLU layer 0 for instance ib: alpha, beta and the optional g / ghat sums.
__device__ __forceinline__ void bottom_reduce_neuron(const BottomArgs& a, int ib, const InstDesc& in, int j,
                                                     double n_rows, const double* s_X) {
    const int d1 = a.d1, d0 = a.d0;
    const int c0 = a.ichunk0[ib], c1 = a.ichunk1[ib];
    const long so = (long)in.slot * a.ld_state + j;
    const int sj = (int)a.S[so];
    // unstable exactly where the fold used the triangle (same test as the kernel)
    const float l = a.l[so], u = a.u[so];
    const bool unst = sj == 0 && !(l >= 0.f) && !(u <= 0.f) && (-(u * l) / (u - l)) > 0.f;
    const bool need_h = a.gsum_hat || sj != 0;
    float da = 0.f, sg = 0.f;
#pragma unroll 4
    for (int c = c0; c < c1; ++c) {
        const float* pt = a.part + (long)c * (2 * d1 + d0);
        if (unst) da += pt[j];
        if (a.gsum_out) sg += pt[d1 + j];
    }
    float sh = 0.f;
    if (need_h) {
        const int HoWo = a.Ho * a.Wo, kk = a.k * a.k;
        const int co = j / HoWo, q = j - co * HoWo, y = q / a.Wo, x = q - y * a.Wo;
        const int Y0 = a.s * y - a.p, X0 = a.s * x - a.p;
        const float* w = a.W1 + (long)co * a.Ci * kk;
        double acc = n_rows * (double)a.b1[co];
        for (int ci = 0; ci < a.Ci; ++ci)
            for (int ky = 0; ky < a.k; ++ky) {
                const int Y = Y0 + ky;
                if ((unsigned)Y >= (unsigned)a.Hi) continue;
                for (int kx = 0; kx < a.k; ++kx) {
                    const int X = X0 + kx;
                    if ((unsigned)X >= (unsigned)a.Wi) continue;
                    acc += (double)w[(ci * a.k + ky) * a.k + kx] * s_X[(ci * a.Hi + Y) * a.Wi + X];
                }
            }
        sh = (float)acc;
    }
    const long go = (long)ib * a.ldg + j;
    a.d_alpha[go] = da;
    a.d_beta[go] = (float)sj * sh;
    if (a.gsum_hat) a.gsum_hat[(long)ib * a.d1 + j] = sh;
    if (a.gsum_out) a.gsum_out[(long)ib * a.d1 + j] = sg;
}

// One workgroup per instance: the sum of x* over the instance's rows is formed once (from the
// chunks' counts of x* = hi), then every neuron's gradients.
constexpr int RDT = 1024;
__global__ __launch_bounds__(RDT) void k_bottom_reduce(BottomArgs a) {
    extern __shared__ double s_X[];   // [d0]
    const int ib = blockIdx.x;
    const InstDesc in = a.inst[ib];
    const int d1 = a.d1, d0 = a.d0;
    const int c0 = a.ichunk0[ib], c1 = a.ichunk1[ib];
    const double n_rows = (double)(in.r1 - in.r0);
    const float* lo = a.lo + (long)a.qid[in.slot] * d0;
    const float* hi = a.hi + (long)a.qid[in.slot] * d0;
    for (int o = threadIdx.x; o < d0; o += RDT) {
        float m = 0.f;   // integer counts: exact in float
#pragma unroll 4
        for (int c = c0; c < c1; ++c) m += a.part[(long)c * (2 * d1 + d0) + 2 * d1 + o];
        s_X[o] = (double)m * (double)hi[o] + (n_rows - (double)m) * (double)lo[o];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < d1; j += RDT) bottom_reduce_neuron(a, ib, in, j, n_rows, s_X);
}

bool bottom_supported(int d1, int d0, int n_weights) {
    // worst-case LDS without the optional MFMA buffers: relaxation and box (up to 6 owned
    // neurons per thread), ahat, g sums, x*, x* counts, weights and bias
    const size_t rxl = cdiv(d1, BT) <= 6 ? 4 * (size_t)d1 + 2 * (size_t)d0 : 0;
    return d1 <= NJ_MAX * BT && d0 <= NO * BT && n_weights <= 4096 &&
           (rxl + 2 * (size_t)d1 + 2 * (size_t)d0 + n_weights + 128) * sizeof(float) <= 150 * 1024;
}

template <bool SRC1>
static void launch_bottom_nj(const BottomArgs& a, int n_blk, size_t lds, hipStream_t st) {
    const int nj = cdiv(a.d1, BT);
    if (nj <= 2)
        hipLaunchKernelGGL((k_bottom<2, SRC1>), dim3(n_blk), dim3(BT), lds, st, a);
    else if (nj <= 4)
        hipLaunchKernelGGL((k_bottom<4, SRC1>), dim3(n_blk), dim3(BT), lds, st, a);
    else if (nj <= 6)
        hipLaunchKernelGGL((k_bottom<6, SRC1>), dim3(n_blk), dim3(BT), lds, st, a);
    else
        hipLaunchKernelGGL((k_bottom<8, SRC1>), dim3(n_blk), dim3(BT), lds, st, a);
}

void launch_bottom(const BottomArgs& a, int n_inst, hipStream_t st) {
    if (n_inst <= 0) return;
    MNB_CHECK(bottom_supported(a.d1, a.d0, a.Co * a.Ci * a.k * a.k) && a.k <= 3 * a.s && (a.s >= 2 || a.k <= 3),
              MNB_EDEVICE, "bottom kernel: unsupported shape");
    const int nb = a.n_chunk;
    if (nb <= 0) return;
    if (bottom_mf_supported(a.Co, a.Ci, a.k, a.s, a.Ho, a.Wo, a.d0, a.d1, a.gsum_out != nullptr) &&
        !(kernel_variants() & MNB_VAR_VALU_BOTTOM)) {
        launch_bottom_mf(a, st);
        return;
    }
    // LDS: relaxation (up to 6 owned neurons per thread), ahat, x*, x* counts, bias,
    // weights (+ g sums with MNCs), and the box when it fits
    const size_t rxl = cdiv(a.d1, BT) <= 6 ? 4 * (size_t)a.d1 : 0;
    const size_t base = (size_t)(a.d1 + 2 * a.d0 + ((a.Co + 3) & ~3) + ((a.Co * a.Ci * a.k * a.k + 3) & ~3) +
                                 (a.gsum_out ? a.d1 : 0));
    MNB_CHECK((base + rxl) * sizeof(float) <= 150 * 1024, MNB_EDEVICE, "bottom kernel: LDS");
    size_t lds = (base + rxl) * sizeof(float);
    BottomArgs b = a;
    b.box_lds = lds + 2 * (size_t)a.d0 * sizeof(float) <= 150 * 1024;
    MNB_CHECK(b.box_lds || !rxl, MNB_EDEVICE, "bottom kernel: LDS");
    if (b.box_lds) lds += 2 * (size_t)a.d0 * sizeof(float);
    if (a.src_mode == 0)
        launch_bottom_nj<false>(b, nb, lds, st);
    else
        launch_bottom_nj<true>(b, nb, lds, st);
    MNB_HIP(hipGetLastError());
}

void launch_bottom_reduce(const BottomArgs& a, int n_inst, hipStream_t st) {
    if (!a.adjoint || n_inst <= 0 || a.n_chunk <= 0) return;
    hipLaunchKernelGGL(k_bottom_reduce, dim3(n_inst), dim3(RDT), (size_t)a.d0 * sizeof(double), st, a);
    MNB_HIP(hipGetLastError());
}

}  // namespace mnb
