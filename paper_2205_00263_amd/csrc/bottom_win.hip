// Window-sparse bottom of the intermediate-bound passes whose objective is ReLU
// layer 1 fed by a convolution of ReLU layer 0's output (the second convolution
// of ConvSmall, the first block convolution of the ResNets).
//
// The row +-e_j on that convolution's output has nonzero coefficients on ReLU
// layer 0 only inside j's filter window (C1 x ok x ok entries).  After the
// ReLU-0 fold (Eq. 5) and the transposed first convolution (Eq. 2) its input
// coefficients are nonzero only on the window's receptive field, apart from
// the split terms S beta of ReLU layer 0, which are the same for every row of
// an instance.  The transposed convolution is linear, so those terms are
// folded once per instance (k_win_prep) into an input-space coefficient A_s,
// its concretisation and its constant; each row then adds only its window.
//
// A workgroup owns one (instance, window position of the objective output):
// all its rows share one window, so the alpha gradient of a window entry
// accumulates in one thread in row order.  The beta gradient of a split neuron
// is S_jj times the sum over rows of ghat_j, the first convolution of x* plus
// bias, which is linear in x*: only the sum of the rows' x* is needed
// (k_win_reduce).  All sums run in a fixed order.
#include "bottom.h"
#include "../../include/mnbab.h"

namespace mnb {

namespace {

constexpr int WT = 256;
typedef float f4 __attribute__((ext_vector_type(4)));

// Fixed-order sum of three per-thread values over a 256-thread block.
__device__ __forceinline__ void win_sum3(float& x, float& y, float& z, float (*red)[4]) {
    x = wave_sum(x);
    y = wave_sum(y);
    z = wave_sum(z);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = x;
        red[1][w] = y;
        red[2][w] = z;
    }
    __syncthreads();
    x = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    y = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    z = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
}

// Per instance: A_s = transposed first convolution of S beta (ReLU layer 0),
// its concretisation sum, |A_s| max(|lo|,|hi|) sum and the constant S beta . bias.
__global__ __launch_bounds__(WT) void k_win_prep(WinArgs a) {
    extern __shared__ float sm[];
    float* s_as = sm;             // [d1]
    float* s_w = s_as + a.d1;     // [C1 * N]
    __shared__ float red[3][4];
    const InstDesc in = a.inst[blockIdx.x];
    const int t = threadIdx.x;
    const int N = a.Ci * a.k * a.k;
    const int HoWo = a.Ho * a.Wo, HiWi = a.Hi * a.Wi;
    for (int i = t; i < a.C1 * N; i += WT) s_w[i] = a.W1[i];
    float cs = 0.f;
    int any = 0;
    const long po = ((long)in.slot * a.n_sets + in.set) * a.ld_param;
    for (int j = t; j < a.d1; j += WT) {
        const int sj = (int)a.S[(long)in.slot * a.ld_state + j];
        const float v = sj != 0 ? (float)sj * a.beta[po + j] : 0.f;
        s_as[j] = v;
        cs += v * a.b1[j / HoWo];
        any |= v != 0.f;
    }
    const int nz = __syncthreads_or(any);
    const int qi = a.qid[in.slot];
    const float* lo = a.lo + (long)qi * a.d0;
    const float* hi = a.hi + (long)qi * a.d0;
    float* As = a.asplit + (long)blockIdx.x * a.d0;
    float L = 0.f, MG = 0.f;
    for (int o = t; o < a.d0; o += WT) {
        float acc = 0.f;
        if (nz) {
            const int ci = o / HiWi, qq = o - ci * HiWi;
            const int Yp = qq / a.Wi + a.p, Xp = qq - (qq / a.Wi) * a.Wi + a.p;
            for (int ky = Yp % a.s; ky < a.k; ky += a.s) {
                const int Y = (Yp - ky) / a.s;
                if (Yp < ky || Y >= a.Ho) continue;
                for (int kx = Xp % a.s; kx < a.k; kx += a.s) {
                    const int X = (Xp - kx) / a.s;
                    if (Xp < kx || X >= a.Wo) continue;
                    for (int c1 = 0; c1 < a.C1; ++c1)
                        acc += s_as[c1 * HoWo + Y * a.Wo + X] * s_w[c1 * N + (ci * a.k + ky) * a.k + kx];
                }
            }
        }
        As[o] = acc;
        const float l = lo[o], h = hi[o];
        L += fminf(acc * l, acc * h);
        MG += fabsf(acc) * fmaxf(fabsf(l), fabsf(h));
    }
    win_sum3(L, MG, cs, red);
    if (t == 0) {
        float* sc = a.scal + (long)blockIdx.x * 4;
        sc[0] = L;
        sc[1] = MG;
        sc[2] = cs;
        sc[3] = 0.f;
    }
}

// NT: 16-wide tap tiles of the first convolution (1: Ci k k <= 16, 2: <= 32).
template <int NT>
__global__ __launch_bounds__(WT) void k_bottom_win(WinArgs a) {
    __shared__ float s_w[16 * 32];    // W1 [c1][tap], taps padded to 32
    __shared__ float s_ah[16 * 16];   // ahat [c1][pos], positions padded to 16
    __shared__ float s_T[16 * 32];    // [pos][tap] tap products of the transposed convolution
    __shared__ float s_x[WT];         // x* on the input window (0 outside the image)
    __shared__ float s_g[16 * 16];    // ghat [c1][pos]
    __shared__ int s_rows[64];
    __shared__ RowDesc s_rd[64];      // the window's row descriptors,
    __shared__ float s_cb[64];        // objective biases (signed)
    __shared__ float s_old[64];       // and previous bounds (mode 0)
    __shared__ int s_cnt[4];
    __shared__ float red[3][4];
    const int w = blockIdx.x, ib = blockIdx.y;
    const InstDesc in = a.inst[ib];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
    const int nwin = a.oHo * a.oWo;
    const int wy = w / a.oWo, wx = w - wy * a.oWo;
    const int P = a.ok * a.ok, E = a.C1 * P;
    const int N = a.Ci * a.k * a.k, kk = a.k * a.k;
    const int IH = (a.ok - 1) * a.s + a.k, IH2 = IH * IH;
    const int NPIX = a.Ci * IH2;
    const int Yb = a.os * wy - a.op, Xb = a.os * wx - a.op;   // window origin on ReLU layer 0
    const int Ib = a.s * Yb - a.p, Jb = a.s * Xb - a.p;       // input-window origin
    const int HoWo = a.Ho * a.Wo, HiWi = a.Hi * a.Wi;
    for (int i = t; i < 16 * 32; i += WT) {
        const int c1 = i >> 5, tap = i & 31;
        s_w[i] = tap < N ? a.W1[c1 * N + tap] : 0.f;
    }
    s_ah[t] = 0.f;
    __syncthreads();

    // ---- this window's rows of the instance, in row order (at most one per output channel)
    int nrows = 0;
    for (int base = in.r0; base < in.r1; base += WT) {
        const int r = base + t;
        const bool m = r < in.r1 && (a.rows[r].j % nwin) == w;
        const unsigned long long bal = __ballot(m);
        if (lane == 0) s_cnt[wave] = __popcll(bal);
        __syncthreads();
        int off = nrows;
        for (int v = 0; v < wave; ++v) off += s_cnt[v];
        const int pos = off + __popcll(bal & ((1ull << lane) - 1ull));
        if (m && pos < 64) s_rows[pos] = r;
        nrows += (s_cnt[0] + s_cnt[1]) + (s_cnt[2] + s_cnt[3]);
        __syncthreads();
    }
    nrows = nrows < 64 ? nrows : 64;
    // per row, loaded once: descriptor, signed objective bias and previous bound (each
    // (slot, neuron) of the objective layer has exactly one row in a pass)
    if (t < nrows) {
        const RowDesc rd = a.rows[s_rows[t]];
        s_rd[t] = rd;
        s_cb[t] = (float)rd.sign * a.bobj[rd.j];
        float old = 0.f;
        if (a.mode == 0) {
            const long e = (long)in.slot * a.ld_state + a.state_off_obj + rd.j;
            old = rd.sign > 0 ? a.lw[e] : a.uw[e];
        }
        s_old[t] = old;
    }

    // ---- window entry e = t: neuron (c1, Yb+dy, Xb+dx) of ReLU layer 0 and its relaxation
    const int c1 = t / P, pe = t - c1 * P, dy = pe / a.ok, dx = pe - dy * a.ok;
    const int Y = Yb + dy, X = Xb + dx;
    const bool ev = t < E && Y >= 0 && Y < a.Ho && X >= 0 && X < a.Wo;
    float dp = 0.f, dn = 0.f, bn = 0.f, b1e = 0.f;
    if (ev) {
        const int j = c1 * HoWo + Y * a.Wo + X;
        const long so = (long)in.slot * a.ld_state + j;
        const float l = a.l[so], u = a.u[so];
        const int sj = (int)a.S[so];
        if (sj == -1) {
            dp = dn = 1.f;
        } else if (sj == 1) {
        } else if (l >= 0.f) {
            dp = dn = 1.f;
        } else if (u <= 0.f) {
        } else {
            dp = a.alpha[((long)in.slot * a.n_sets + in.set) * a.ld_param + j];
            const float wd = u - l;
            dn = u / wd;
            bn = -(u * l) / wd;
        }
        b1e = a.b1[c1];
    }
    // ---- input-window pixel q = t: (ciq, Ib+qy, Jb+qx)
    const int ciq = t / IH2, rq = t - ciq * IH2, qy = rq / IH, qx = rq - qy * IH;
    const int py = Ib + qy, px = Jb + qx;
    const bool qv = t < NPIX && py >= 0 && py < a.Hi && px >= 0 && px < a.Wi;
    float lo_q = 0.f, hi_q = 0.f, as_q = 0.f;
    if (qv) {
        const long o = (long)ciq * HiWi + py * a.Wi + px;
        const long qo = (long)a.qid[in.slot] * a.d0;
        lo_q = a.lo[qo + o];
        hi_q = a.hi[qo + o];
        as_q = a.asplit[(long)ib * a.d0 + o];
    }
    // split terms outside the window: the instance totals minus the window's share
    float Lw = qv ? fminf(as_q * lo_q, as_q * hi_q) : 0.f;
    float Mw = qv ? fabsf(as_q) * fmaxf(fabsf(lo_q), fabsf(hi_q)) : 0.f;
    float zz = 0.f;
    win_sum3(Lw, Mw, zz, red);
    const float* sc = a.scal + (long)ib * 4;
    const float L_out = sc[0] - Lw, M_out = sc[1] - Mw, c_split = sc[2];

    // ---- MFMA operands held in registers
    const int nt = wave < NT ? wave : NT - 1;
    float bT[4];   // transposed: B[k = c1][n = tap]
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) bT[ks] = s_w[(ks * 4 + lk) * 32 + nt * 16 + lr];
    float bF[8];   // adjoint: B[k = tap][n = c1]
    int xi[8];     // adjoint A operand: s_x index of (pos = lr, tap = 4 ks + lk), -1 if none
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        const int tap = ks * 4 + lk;
        bF[ks] = s_w[lr * 32 + tap];
        int idx = -1;
        if (tap < N && lr < P) {
            const int ci = tap / kk, rr = tap - ci * kk, ky = rr / a.k, kx = rr - ky * a.k;
            const int pdy = lr / a.ok, pdx = lr - pdy * a.ok;
            idx = (ci * IH + a.s * pdy + ky) * IH + a.s * pdx + kx;
        }
        xi[ks] = idx;
    }
    const float b1_lane = a.b1[lr];
    __syncthreads();   // red[] is reused by the rows; s_rd, s_cb, s_old are visible
    // objective filter entry of the next row, loaded one row ahead
    float wnext = (ev && nrows > 0) ? a.Wobj[(long)(s_rd[0].j / nwin) * E + t] : 0.f;

    float da = 0.f, xs = 0.f;
    for (int ri = 0; ri < nrows; ++ri) {
        const int r = s_rows[ri];
        const RowDesc rd = s_rd[ri];
        const float sgn = (float)rd.sign;
        const float wcur = wnext;
        if (ev && ri + 1 < nrows) wnext = a.Wobj[(long)(s_rd[ri + 1].j / nwin) * E + t];
        // fold of ReLU layer 0 on the window (Eq. 5); S beta is in the instance terms
        float ap = 0.f, ce = 0.f;
        if (ev) {
            ap = sgn * wcur;
            const bool neg = ap < 0.f;
            const float ah = ap * (neg ? dn : dp);
            s_ah[c1 * 16 + pe] = ah;
            ce = (neg ? ap * bn : 0.f) + ah * b1e;
        }
        __syncthreads();
        // transposed first convolution on the window: T[pos][tap] = sum_c1 ahat[c1][pos] W1[c1][tap]
        if (wave < NT) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(s_ah[(ks * 4 + lk) * 16 + lr], bT[ks], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) s_T[(4 * lk + v) * 32 + nt * 16 + lr] = acc[v];
        }
        __syncthreads();
        // col2im onto the input window plus A_s, then concretisation over the box (Eq. 6)
        float lbp = 0.f, mag = 0.f, xq = 0.f;
        if (qv) {
            float acc = as_q;
            for (int ky = qy % a.s; ky < a.k; ky += a.s) {
                const int pdy = (qy - ky) / a.s;
                if (qy < ky || pdy >= a.ok) continue;
                for (int kx = qx % a.s; kx < a.k; kx += a.s) {
                    const int pdx = (qx - kx) / a.s;
                    if (qx < kx || pdx >= a.ok) continue;
                    acc += s_T[(pdy * a.ok + pdx) * 32 + (ciq * a.k + ky) * a.k + kx];
                }
            }
            lbp = fminf(acc * lo_q, acc * hi_q);
            mag = fabsf(acc) * fmaxf(fabsf(lo_q), fabsf(hi_q));
            xq = acc < 0.f ? hi_q : lo_q;
        }
        s_x[t] = xq;
        win_sum3(lbp, mag, ce, red);   // also publishes s_x
        if (t == 0) {
            const float cpt = (ce + c_split) + s_cb[ri];
            float lb = ((L_out + lbp) + cpt) - ((M_out + mag) + fabsf(cpt)) * 9.5367431640625e-07f;   // 2^-20 margin
            if (!(lb == lb) || isinf(lb)) lb = -INFINITY;
            if (a.mode == 0) {
                const long e = (long)in.slot * a.ld_state + a.state_off_obj + rd.j;
                if (rd.sign > 0)
                    a.lw[e] = fmaxf(s_old[ri], lb);
                else
                    a.uw[e] = fminf(s_old[ri], isinf(lb) ? INFINITY : -lb);
            } else {
                a.lb_out[r] = lb;
            }
        }
        if (a.adjoint) {
            // ghat on the window: im2col(x*) W1^T plus bias
            if (wave == 0) {
                f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) {
                    if (ks * 4 >= N) break;
                    const float av = xi[ks] >= 0 ? s_x[xi[ks]] : 0.f;
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bF[ks], acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) s_g[lr * 16 + 4 * lk + v] = acc[v] + b1_lane;
            }
            __syncthreads();
            if (ev && bn > 0.f && !(ap < 0.f)) da += ap * s_g[c1 * 16 + pe];
            xs += xq;
        }
        vmem_drain();      // the next row's filter entry has arrived; nothing left in flight
        __syncthreads();   // s_ah, s_T, s_x, s_g and red[] are rewritten by the next row
    }
    if (!a.adjoint) return;
    const long blk = (long)ib * nwin + w;
    if (t < E) a.part_a[blk * E + t] = da;
    if (t < NPIX) a.part_x[blk * NPIX + t] = qv ? xs - (float)nrows * (as_q < 0.f ? hi_q : lo_q) : 0.f;
    if (t == 0) a.part_n[blk] = nrows;
}

// Instance gradients: alpha from the window partials (windows in order), beta from the
// first convolution of the instance's x* sum.
__global__ __launch_bounds__(WT) void k_win_reduce(WinArgs a) {
    extern __shared__ float sm[];
    float* s_X = sm;              // [d0]
    float* s_w = s_X + a.d0;      // [C1 * N]
    const int ib = blockIdx.x;
    const InstDesc in = a.inst[ib];
    const int t = threadIdx.x;
    const int nwin = a.oHo * a.oWo;
    const int P = a.ok * a.ok, E = a.C1 * P;
    const int N = a.Ci * a.k * a.k;
    const int IH = (a.ok - 1) * a.s + a.k;
    const int NPIX = a.Ci * IH * IH;
    const int HoWo = a.Ho * a.Wo, HiWi = a.Hi * a.Wi;
    for (int i = t; i < a.C1 * N; i += WT) s_w[i] = a.W1[i];
    int ntot = 0;
    for (int w = 0; w < nwin; ++w) ntot += a.part_n[(long)ib * nwin + w];
    const long qo = (long)a.qid[in.slot] * a.d0;
    for (int o = t; o < a.d0; o += WT) {
        const int ci = o / HiWi, qq = o - ci * HiWi, py = qq / a.Wi, px = qq - py * a.Wi;
        const float as = a.asplit[(long)ib * a.d0 + o];
        float Xs = (float)ntot * (as < 0.f ? a.hi[qo + o] : a.lo[qo + o]);
        for (int wy = 0; wy < a.oHo; ++wy) {
            const int qy = py - (a.s * (a.os * wy - a.op) - a.p);
            if (qy < 0 || qy >= IH) continue;
            for (int wx = 0; wx < a.oWo; ++wx) {
                const int qx = px - (a.s * (a.os * wx - a.op) - a.p);
                if (qx < 0 || qx >= IH) continue;
                Xs += a.part_x[((long)ib * nwin + wy * a.oWo + wx) * NPIX + (ci * IH + qy) * IH + qx];
            }
        }
        s_X[o] = Xs;
    }
    __syncthreads();
    for (int j = t; j < a.d1; j += WT) {
        const int c1 = j / HoWo, qq = j - c1 * HoWo, Y = qq / a.Wo, X = qq - Y * a.Wo;
        const long so = (long)in.slot * a.ld_state + j;
        const int sj = (int)a.S[so];
        const float l = a.l[so], u = a.u[so];
        // unstable exactly where the fold used the triangle (same test as the kernel)
        const bool unst = sj == 0 && !(l >= 0.f) && !(u <= 0.f) && (-(u * l) / (u - l)) > 0.f;
        float dal = 0.f;
        if (unst) {
            for (int wy = 0; wy < a.oHo; ++wy) {
                const int dy = Y - (a.os * wy - a.op);
                if (dy < 0 || dy >= a.ok) continue;
                for (int wx = 0; wx < a.oWo; ++wx) {
                    const int dx = X - (a.os * wx - a.op);
                    if (dx < 0 || dx >= a.ok) continue;
                    dal += a.part_a[((long)ib * nwin + wy * a.oWo + wx) * E + c1 * P + dy * a.ok + dx];
                }
            }
        }
        float dbe = 0.f;
        if (sj != 0) {
            float g = (float)ntot * a.b1[c1];
            for (int ci = 0; ci < a.Ci; ++ci)
                for (int ky = 0; ky < a.k; ++ky) {
                    const int yy = a.s * Y - a.p + ky;
                    if (yy < 0 || yy >= a.Hi) continue;
                    for (int kx = 0; kx < a.k; ++kx) {
                        const int xx = a.s * X - a.p + kx;
                        if (xx < 0 || xx >= a.Wi) continue;
                        g += s_w[c1 * N + (ci * a.k + ky) * a.k + kx] * s_X[ci * HiWi + yy * a.Wi + xx];
                    }
                }
            dbe = (float)sj * g;
        }
        a.d_alpha[(long)ib * a.ldg + j] = dal;
        a.d_beta[(long)ib * a.ldg + j] = dbe;
    }
}

}  // namespace

bool win_supported(int C1, int Ci, int k, int s, int ok, int oCo, int d1, int d0) {
    const int IH = (ok - 1) * s + k;
    return C1 == 16 && ok * ok <= 16 && Ci * IH * IH <= WT && Ci * k * k <= 32 && oCo <= 64 &&
           (size_t)(d1 + 16 * 32) * sizeof(float) <= 64 * 1024 && (size_t)(d0 + 16 * 32) * sizeof(float) <= 64 * 1024;
}

void launch_bottom_win(const WinArgs& a, int n_inst, hipStream_t st) {
    if (n_inst <= 0) return;
    MNB_CHECK(win_supported(a.C1, a.Ci, a.k, a.s, a.ok, a.oCo, a.d1, a.d0) && a.oCi == a.C1 &&
                  a.oHi == a.Ho && a.oWi == a.Wo && (a.mode == 0 || a.mode == 2),
              MNB_EDEVICE, "window bottom kernel: unsupported shape");
    MNB_CHECK(n_inst <= 65535, MNB_EDEVICE, "window bottom kernel: too many instances in one pass");
    const int N = a.Ci * a.k * a.k;
    hipLaunchKernelGGL(k_win_prep, dim3(n_inst), dim3(WT), (a.d1 + a.C1 * N) * sizeof(float), st, a);
    MNB_HIP(hipGetLastError());
    const dim3 grid(a.oHo * a.oWo, n_inst);
    if (N <= 16)
        hipLaunchKernelGGL(k_bottom_win<1>, grid, dim3(WT), 0, st, a);
    else
        hipLaunchKernelGGL(k_bottom_win<2>, grid, dim3(WT), 0, st, a);
    MNB_HIP(hipGetLastError());
}

void launch_bottom_win_reduce(const WinArgs& a, int n_inst, hipStream_t st) {
    if (!a.adjoint || n_inst <= 0) return;
    const int N = a.Ci * a.k * a.k;
    hipLaunchKernelGGL(k_win_reduce, dim3(n_inst), dim3(WT), (a.d0 + a.C1 * N) * sizeof(float), st, a);
    MNB_HIP(hipGetLastError());
}

}  // namespace mnb
