// Fused bottom of a back-substitution pass on v_mfma_f32_16x16x4_f32, for networks
// whose first layer is a convolution into 16 channels with at most 32 taps per
// channel (ConvSmall, the ResNet stems).
//
// One workgroup owns one chunk of rows of one instance (subproblem, parameter
// set).  The positions of ReLU layer 0 are cut into 16-position tiles; each of the
// 16 wavefronts owns one tile (TPW), and in a tile lane (lr, lk) owns the four
// neurons (channel 4 lk + v, position 16 mt + lr), v = 0..3, for the whole chunk.
// Per row:
//   fold of ReLU layer 0 (Eq. 5) in registers: a' -> ahat
//   transposed first convolution (Eq. 2): T[pos][tap] = sum_co ahat[co][pos] W[co][tap],
//       with ahat as the MFMA A operand straight from registers    -> T in LDS
//   barrier; col2im of T, concretisation over the box (Eq. 6), x*   -> x* in LDS
//   block reduction of the bound (barrier)
//   adjoint: ghat^T[co][pos] = sum_tap W[co][tap] x*[pos][tap] + b, whose MFMA
//       output lands in the lanes that hold a' for the same neurons, so the
//       relaxation of ReLU layer 0, the alpha-gradient sums and the rows' g are
//       computed in registers.
// Two barriers per row.  The alpha sums run over the chunk's rows in order; the
// ghat sums for beta come from per-element counts of x* = hi (k_bottom_reduce).
#include "bottom.h"
#include "../../include/mnbab.h"

namespace mnb {

namespace {

constexpr int MBT = 1024;        // threads (16 wavefronts, one 16-position tile each)
constexpr int MNW = MBT / 64;
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum of three per-thread values over the block (fixed order); one barrier.
__device__ __forceinline__ void bsum3(float& x, float& y, float& z, float (*red)[MNW]) {
    x = wave_sum(x);
    y = wave_sum(y);
    z = wave_sum(z);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = x;
        red[1][w] = y;
        red[2][w] = z;
    }
    lds_sync();
    float v[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float* rq = red[q];
        const float h0 = ((rq[0] + rq[1]) + (rq[2] + rq[3])) + ((rq[4] + rq[5]) + (rq[6] + rq[7]));
        const float h1 = ((rq[8] + rq[9]) + (rq[10] + rq[11])) + ((rq[12] + rq[13]) + (rq[14] + rq[15]));
        v[q] = h0 + h1;
    }
    x = v[0];
    y = v[1];
    z = v[2];
}

// TPW: tiles per wavefront (1 is instantiated: up to 16 tiles); KK, SS: kernel size and
// stride as constants (0: runtime); NTT: 16-tap tiles of the first convolution (1: at most
// 16 taps, 2: at most 32); SRC1: rows built from the objective convolution's filter;
// O1: at most one input element per thread (d0 <= 1024), whose col2im taps and box are
// then held in registers for the whole chunk.
template <int TPW, int KK, int SS, int NTT, bool SRC1, bool O1>
__global__ __launch_bounds__(MBT) void k_bottom_mf(BottomArgs a) {
    constexpr int KSM = 4 * NTT;   // 4-tap steps of the adjoint product
    const int k = KK ? KK : a.k;
    const int s = SS ? SS : a.s;
    const int d1 = a.d1, d0 = a.d0;
    const int HoWo = a.Ho * a.Wo, HiWi = a.Hi * a.Wi;
    const int kk = k * k, ntap = a.Ci * kk;
    const int MT = (HoWo + 15) >> 4;
    extern __shared__ float smem[];
    float* s_T = smem;                                   // [16 NTT][HoWo] tap products, tap-major
    float* s_x = s_T + 16 * NTT * HoWo;                  // [d0] x* of the current row
    int* s_xc = reinterpret_cast<int*>(s_x + d0);        // [d0] rows of the chunk with x*_o = hi_o
    float* s_lo = s_x + 2 * d0;                          // [d0] box (box_lds)
    float* s_hi = s_lo + d0;                             // [d0]
    float* s_sg = s_x + 2 * d0 + (a.box_lds ? 2 * d0 : 0);   // [d1] sum of g (MNC only)
    __shared__ float red[3][MNW];
    __shared__ RowDesc s_rd[BOTTOM_CHUNK_ROWS];
    __shared__ float s_crow[BOTTOM_CHUNK_ROWS];
    __shared__ float s_old[BOTTOM_CHUNK_ROWS];

    const int ib = a.cinst[blockIdx.x];
    const InstDesc in = a.inst[ib];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
    // the chunk's rows (at most BOTTOM_CHUNK_ROWS by construction of the chunks): descriptor,
    // constant and previous bound of each, loaded once with all loads in flight together
    const int cr0 = a.cr0[blockIdx.x];
    const int nr = min(a.cr1[blockIdx.x] - cr0, BOTTOM_CHUNK_ROWS);
    for (int ri = wave; ri < nr; ri += MNW) {
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
    const float* glo = a.lo + (long)a.qid[in.slot] * d0;
    const float* ghi = a.hi + (long)a.qid[in.slot] * d0;
    float b1v[4];   // bias of the owned channels 4 lk + v
#pragma unroll
    for (int v = 0; v < 4; ++v) b1v[v] = a.b1[4 * lk + v];
    // O1: the owned input element o = t, its tap products in s_T (-1: none) and its box
    constexpr int NTO = KK ? ((KK + SS - 1) / SS) * ((KK + SS - 1) / SS) : 9;
    int tix[O1 ? NTO : 1];
    float lo_o = 0.f, hi_o = 0.f;
    if constexpr (O1) {
        const bool ov = t < d0;
        const int o = ov ? t : 0;
        const int ci = o / HiWi, qq = o - ci * HiWi;
        const int Yq = qq / a.Wi;
        const int Yp = Yq + a.p, Xp = qq - Yq * a.Wi + a.p;
        const int nty = (k + s - 1) / s;
#pragma unroll
        for (int q = 0; q < NTO; ++q) {
            const int ty = q / (KK ? (KK + SS - 1) / SS : 3), tx = q - ty * (KK ? (KK + SS - 1) / SS : 3);
            const int ky = Yp % s + ty * s, kx = Xp % s + tx * s;
            const int y = (Yp - ky) / s, x = (Xp - kx) / s;
            const bool tv = ov && ty < nty && tx < nty && ky < k && kx < k && Yp >= ky && Xp >= kx && y < a.Ho && x < a.Wo;
            tix[q] = tv ? ((ci * k + ky) * k + kx) * HoWo + y * a.Wo + x : -1;
        }
        if (ov) {
            lo_o = glo[o];
            hi_o = ghi[o];
        }
    }
    for (int o = t; o < d0; o += MBT) {
        s_xc[o] = 0;
        if (a.box_lds) {
            s_lo[o] = glo[o];
            s_hi[o] = ghi[o];
        }
    }
    if (a.gsum_out)
        for (int j = t; j < d1; j += MBT) s_sg[j] = 0.f;

    // first-layer weights as MFMA operands held for the whole chunk:
    // transposed product B[k = co][n = tap] with co = 4 lk + ks, tap = 16 nt + lr;
    // adjoint product A[m = co][k = tap] with co = lr, tap = 4 ks + lk
    float bT[NTT][4], aW[KSM];
#pragma unroll
    for (int nt = 0; nt < NTT; ++nt)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int tap = nt * 16 + lr;
            bT[nt][ks] = tap < ntap ? a.W1[(4 * lk + ks) * ntap + tap] : 0.f;
        }
#pragma unroll
    for (int ks = 0; ks < KSM; ++ks) {
        const int tap = 4 * ks + lk;
        aW[ks] = tap < ntap ? a.W1[lr * ntap + tap] : 0.f;
    }

    // owned neurons: tile mt = wave + u MNW, neuron (co = 4 lk + v, pos = 16 mt + lr)
    // relaxation of ReLU layer 0 (split first, then stable, then unstable): slope where
    // a' >= 0, slope and intercept where a' < 0 (the intercept is > 0 exactly when
    // unstable), S beta + (Phat^T gamma)
    float rdp[TPW][4], rdn[TPW][4], rbn[TPW][4], rad[TPW][4];
    int gidx[TPW][KSM];   // adjoint B operand: s_x index of (pos = 16 mt + lr, tap = 4 ks + lk), -1: none
    const long so0 = (long)in.slot * a.ld_state;
    const long po0 = ((long)in.slot * a.n_sets + in.set) * a.ld_param;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int pos = (wave + u * MNW) * 16 + lr;
        const bool pv = pos < HoWo;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = (4 * lk + v) * HoWo + pos;
            float dp = 0.f, dn = 0.f, bn = 0.f, ad = 0.f;
            if (pv) {
                const float l = a.l[so0 + j], uu = a.u[so0 + j];
                const int sj = (int)a.S[so0 + j];
                if (sj == -1) {
                    dp = dn = 1.f;
                } else if (sj == 1) {
                } else if (l >= 0.f) {
                    dp = dn = 1.f;
                } else if (uu <= 0.f) {
                } else {
                    dp = a.alpha[po0 + j];
                    const float w = uu - l;
                    dn = uu / w;
                    bn = -(uu * l) / w;
                }
                ad = (sj != 0 ? (float)sj * a.beta[po0 + j] : 0.f) + (a.vhat ? a.vhat[(long)ib * d1 + j] : 0.f);
            }
            rdp[u][v] = dp;
            rdn[u][v] = dn;
            rbn[u][v] = bn;
            rad[u][v] = ad;
        }
        const int y = pv ? pos / a.Wo : 0, x = pv ? pos - y * a.Wo : 0;
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks) {
            const int tap = 4 * ks + lk;
            int idx = -1;
            if (pv && tap < ntap) {
                const int ci = tap / kk, rr = tap - ci * kk, ky = rr / k, kx = rr - ky * k;
                const int Y = s * y - a.p + ky, X = s * x - a.p + kx;
                if ((unsigned)Y < (unsigned)a.Hi && (unsigned)X < (unsigned)a.Wi) idx = (ci * a.Hi + Y) * a.Wi + X;
            }
            gidx[u][ks] = idx;
        }
    }
    float da[TPW][4];
#pragma unroll
    for (int u = 0; u < TPW; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) da[u][v] = 0.f;
    const float* vrow = a.v ? a.v + (long)ib * d1 : nullptr;
    const float gpv = a.gp ? a.gp[ib] : 0.f;
    // coefficients of the next row, loaded one row ahead (the first row's before the barrier,
    // which waits for them)
    float nx[SRC1 ? 1 : TPW][4];
    if constexpr (!SRC1) {
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int pos = (wave + u * MNW) * 16 + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                nx[u][v] = (pos < HoWo && nr > 0) ? a.A[(long)cr0 * d1 + (4 * lk + v) * HoWo + pos] : 0.f;
        }
    }
    __syncthreads();

    for (int ri = 0; ri < nr; ++ri) {
        const int r = cr0 + ri;
        const RowDesc rd = s_rd[ri];
        // ---- row coefficients a on the owned neurons of ReLU layer 0
        float ap[TPW][4];
        if constexpr (!SRC1) {
#pragma unroll
            for (int u = 0; u < TPW; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) ap[u][v] = nx[u][v];
            if (ri + 1 < nr) {
#pragma unroll
                for (int u = 0; u < TPW; ++u) {
                    const int pos = (wave + u * MNW) * 16 + lr;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        nx[u][v] = pos < HoWo ? a.A[(long)(r + 1) * d1 + (4 * lk + v) * HoWo + pos] : 0.f;
                }
            }
        } else {
            // +-e_j on the output of the objective convolution: its filter placed at j
            const float sgn = (float)rd.sign;
            const int per = a.oHo * a.oWo;
            const int oco = rd.j / per, opos = rd.j - oco * per;
            const int oy = opos / a.oWo, ox = opos - oy * a.oWo;
            const float* wrow = a.Wobj + (long)oco * a.oCi * a.ok * a.ok;
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int pos = (wave + u * MNW) * 16 + lr;
                const int Y = pos < HoWo ? pos / a.oWi : 0, X = pos - Y * a.oWi;
                const int ky = Y - a.os * oy + a.op, kx = X - a.os * ox + a.op;
                const bool in_w = pos < HoWo && (unsigned)ky < (unsigned)a.ok && (unsigned)kx < (unsigned)a.ok;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    ap[u][v] = in_w ? sgn * wrow[((4 * lk + v) * a.ok + ky) * a.ok + kx] : 0.f;
            }
        }
        if (vrow) {
            float vv[TPW][4];
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int pos = (wave + u * MNW) * 16 + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) vv[u][v] = pos < HoWo ? vrow[(4 * lk + v) * HoWo + pos] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < TPW; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) ap[u][v] += vv[u][v];
        }
        // ---- fold of ReLU layer 0 and the transposed first convolution of each owned tile
        float cpt = 0.f;
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int mt = wave + u * MNW;
            float ah[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float p = ap[u][v];
                const bool neg = p < 0.f;
                ah[v] = p * (neg ? rdn[u][v] : rdp[u][v]) + rad[u][v];
                cpt += (neg ? p * rbn[u][v] : 0.f) + ah[v] * b1v[v];
            }
            if (mt < MT) {
#pragma unroll
                for (int nt = 0; nt < NTT; ++nt) {
                    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[ks], bT[nt][ks], acc, 0, 0, 0);
                    // lane holds T[pos = 16 mt + 4 lk + v][tap = 16 nt + lr]
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int p2 = mt * 16 + 4 * lk + v;
                        if (p2 < HoWo) s_T[(nt * 16 + lr) * HoWo + p2] = acc[v];
                    }
                }
            }
        }
        if (a.Ap_out) {
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int pos = (wave + u * MNW) * 16 + lr;
                if (pos < HoWo)
#pragma unroll
                    for (int v = 0; v < 4; ++v) a.Ap_out[(long)r * d1 + (4 * lk + v) * HoWo + pos] = ap[u][v];
            }
        }
        if (t == 0) cpt += s_crow[ri] - gpv;
        lds_sync();
        // ---- col2im onto the input and concretisation over the box (Eq. 6), x*
        float lbp = 0.f, mag = 0.f;
        if constexpr (O1) {
            if (t < d0) {
                float acc = 0.f;
#pragma unroll
                for (int q = 0; q < NTO; ++q)
                    if (tix[q] >= 0) acc += s_T[tix[q]];
                lbp = fminf(acc * lo_o, acc * hi_o);
                mag = fabsf(acc) * fmaxf(fabsf(lo_o), fabsf(hi_o));
                const bool neg = acc < 0.f;
                s_x[t] = neg ? hi_o : lo_o;
                if (a.adjoint && neg) s_xc[t] += 1;
                if (a.xbits) a.xbits[(long)r * d0 + t] = neg ? 1 : 0;
            }
        } else
        for (int o = t; o < d0; o += MBT) {
            const int ci = o / HiWi, qq = o - ci * HiWi;
            const int Yq = qq / a.Wi;
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
                    acc += s_T[((ci * k + ky) * k + kx) * HoWo + y * a.Wo + x];
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
            if (a.adjoint && neg) s_xc[o] += 1;
            if (a.xbits) a.xbits[(long)r * d0 + o] = neg ? 1 : 0;
        }
        bsum3(lbp, mag, cpt, red);   // also publishes s_x
        if (t == 0) {
            float lb = (lbp + cpt) - (mag + fabsf(cpt)) * 9.5367431640625e-07f;   // 2^-20 rounding margin
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
            // ---- adjoint: ghat^T = W1 im2col(x*)^T + b1 per owned tile, then the relaxation of
            // ReLU layer 0 and the alpha (and MNC g) sums of the owned neurons
            float gv[TPW][4];
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int mt = wave + u * MNW;
                f4 acc = {0.f, 0.f, 0.f, 0.f};
                if (mt < MT) {
#pragma unroll
                    for (int ks = 0; ks < KSM; ++ks) {
                        if (4 * ks >= ntap) break;
                        const int gi = gidx[u][ks];
                        const float xv = gi >= 0 ? s_x[gi] : 0.f;
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aW[ks], xv, acc, 0, 0, 0);
                    }
                }
                const int pos = mt * 16 + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    // lane holds ghat[co = 4 lk + v][pos = 16 mt + lr] without the bias
                    const float gh = acc[v] + b1v[v];
                    const float p = ap[u][v];
                    const bool neg = p < 0.f;
                    const float bn = rbn[u][v];
                    const float g = (neg ? rdn[u][v] : rdp[u][v]) * gh + (neg ? bn : 0.f);
                    if (bn > 0.f && !neg) da[u][v] += p * gh;
                    if (a.gsum_out && pos < HoWo) s_sg[(4 * lk + v) * HoWo + pos] += g;
                    gv[u][v] = g;
                }
            }
            vmem_drain();
            if (a.Gout) {
#pragma unroll
                for (int u = 0; u < TPW; ++u) {
                    const int pos = (wave + u * MNW) * 16 + lr;
                    if (pos < HoWo)
#pragma unroll
                        for (int v = 0; v < 4; ++v) a.Gout[(long)r * d1 + (4 * lk + v) * HoWo + pos] = gv[u][v];
                }
            }
        } else {
            vmem_drain();
        }
        // next row: its T writes follow the barrier above (every col2im read is done) and its
        // x* writes follow its first barrier (every adjoint gather of this row is done)
    }
    if (!a.adjoint) return;
    lds_sync();   // s_sg and s_xc complete
    // partial sums of this chunk: alpha only where the neuron is unstable, the g sum only for
    // MNCs, and per input element the number of rows with x* = hi
    float* pt = a.part + (long)blockIdx.x * (2 * d1 + d0);
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int pos = (wave + u * MNW) * 16 + lr;
        if (pos < HoWo)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = (4 * lk + v) * HoWo + pos;
                if (rbn[u][v] > 0.f) pt[j] = da[u][v];
                if (a.gsum_out) pt[d1 + j] = s_sg[j];
            }
    }
    for (int o = t; o < d0; o += MBT) pt[2 * d1 + o] = (float)s_xc[o];
}

template <int TPW, int KK, int SS, int NTT, bool O1>
void launch_mf_o1(const BottomArgs& a, size_t lds, hipStream_t st) {
    if (a.src_mode == 0)
        hipLaunchKernelGGL((k_bottom_mf<TPW, KK, SS, NTT, false, O1>), dim3(a.n_chunk), dim3(MBT), lds, st, a);
    else
        hipLaunchKernelGGL((k_bottom_mf<TPW, KK, SS, NTT, true, O1>), dim3(a.n_chunk), dim3(MBT), lds, st, a);
}

template <int TPW, int KK, int SS, int NTT>
void launch_mf_src(const BottomArgs& a, size_t lds, hipStream_t st) {
    if (a.d0 <= MBT)
        launch_mf_o1<TPW, KK, SS, NTT, true>(a, lds, st);
    else
        launch_mf_o1<TPW, KK, SS, NTT, false>(a, lds, st);
}

template <int KK, int SS, int NTT>
void launch_mf_tpw(const BottomArgs& a, size_t lds, hipStream_t st) {
    launch_mf_src<1, KK, SS, NTT>(a, lds, st);
}

}  // namespace

bool bottom_mf_supported(int Co, int Ci, int k, int Ho, int Wo, int d0, int d1, bool mnc) {
    const int HoWo = Ho * Wo, ntap = Ci * k * k;
    const size_t lds = ((size_t)16 * (ntap > 16 ? 2 : 1) * HoWo + 2 * (size_t)d0 + (mnc ? (size_t)d1 : 0)) * sizeof(float);
    return Co == 16 && ntap <= 32 && (HoWo + 15) / 16 <= MNW && lds <= 150 * 1024;
}

void launch_bottom_mf(const BottomArgs& a, hipStream_t st) {
    const int HoWo = a.Ho * a.Wo, ntap = a.Ci * a.k * a.k;
    MNB_CHECK(bottom_mf_supported(a.Co, a.Ci, a.k, a.Ho, a.Wo, a.d0, a.d1, a.gsum_out != nullptr) && a.d1 == 16 * HoWo,
              MNB_EDEVICE, "bottom kernel (MFMA): unsupported shape");
    const int ntt = ntap > 16 ? 2 : 1;
    size_t lds = ((size_t)16 * ntt * HoWo + 2 * (size_t)a.d0 + (a.gsum_out ? (size_t)a.d1 : 0)) * sizeof(float);
    BottomArgs b = a;
    b.box_lds = lds + 2 * (size_t)a.d0 * sizeof(float) <= 80 * 1024;
    if (b.box_lds) lds += 2 * (size_t)a.d0 * sizeof(float);
    if (ntt == 1 && a.k == 4 && a.s == 2)
        launch_mf_tpw<4, 2, 1>(b, lds, st);
    else if (ntt == 2 && a.k == 3 && a.s == 2)
        launch_mf_tpw<3, 2, 2>(b, lds, st);
    else if (ntt == 1)
        launch_mf_tpw<0, 0, 1>(b, lds, st);
    else
        launch_mf_tpw<0, 0, 2>(b, lds, st);
    MNB_HIP(hipGetLastError());
}

}  // namespace mnb
