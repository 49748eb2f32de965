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
    float L = 0.f, unused = 0.f;
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
    }
    win_sum3(L, unused, cs, red);
    if (t == 0) {
        float* sc = a.scal + (long)blockIdx.x * 4;
        sc[0] = L;
        sc[1] = 0.f;
        sc[2] = cs;
        sc[3] = 0.f;
    }
}

// Rows of each (instance, window position) in pass order: one workgroup per instance
// partitions the instance's rows by the window position of their objective neuron
// (stable, so the order is the pass order and does not depend on the rest of the batch),
// and records with each row its signed objective bias.  The lists depend on the pass's
// rows only, so they are built once for all evaluations of a pass.
__global__ __launch_bounds__(WT) void k_win_rows(WinArgs a) {
    extern __shared__ int s_win[];   // [rows of the instance] window position of each row
    __shared__ int s_pre[65];
    const int ib = blockIdx.x;
    const InstDesc in = a.inst[ib];
    const int t = threadIdx.x;
    const int nwin = a.oHo * a.oWo, n = in.r1 - in.r0;
    for (int i = t; i < n; i += WT) s_win[i] = a.rows[in.r0 + i].j % nwin;
    __syncthreads();
    int cnt = 0;
    if (t < nwin)
        for (int i = 0; i < n; ++i) cnt += s_win[i] == t;
    if (t < nwin) s_pre[t + 1] = cnt;
    __syncthreads();
    if (t == 0) {
        s_pre[0] = 0;
        for (int w = 0; w < nwin; ++w) s_pre[w + 1] += s_pre[w];
    }
    __syncthreads();
    int* ptr = a.win_ptr + (long)ib * (nwin + 1);
    if (t <= nwin) ptr[t] = in.r0 + s_pre[t];
    if (t < nwin) {
        int k = in.r0 + s_pre[t];
        for (int i = 0; i < n; ++i) {
            if (s_win[i] != t) continue;
            const int r = in.r0 + i;
            const RowDesc rd = a.rows[r];
            WinEnt e;
            e.r = rd.sign > 0 ? r : ~r;
            e.j = rd.j;
            e.cb = (float)rd.sign * a.bobj[rd.j];
            e.old = 0.f;
            a.win_ent[k++] = e;
        }
    }
}

// Wavefront-scope ordering of a wavefront's LDS buffers.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// NT: 16-wide tap tiles of the first convolution (1: Ci k k <= 16, 2: <= 32).
// A workgroup owns one (instance, window position); its four wavefronts take the window's
// rows in turn (row i -> wavefront i mod 4), each row end to end without workgroup
// barriers.  Lane (lr, lk) owns the window entries (c1 = 4 lk + v, position lr) through the
// fold, the transposed MFMA (A operand from registers) and the adjoint MFMA, computed as
// ghat^T = W1 im2col(x*)^T so that its output lands in the same lanes; the input-window
// pixels lane + 64 i are owned for col2im and the box.  The alpha and x* sums of each
// wavefront's rows are merged over the wavefronts in a fixed order at the end.
template <int NT>
__global__ __launch_bounds__(WT) void k_bottom_win(WinArgs a) {
    constexpr int NW = WT / 64;
    // per wavefront: T[pos][tap] of the transposed convolution, then one zero (never written: the
    // target of the col2im taps that do not exist)
    constexpr int TZ = 16 * 32;
    __shared__ float s_T[NW][TZ + 1];
    __shared__ float s_x[NW][WT];        // per wavefront: x* on the input window (0 outside the image)
    __shared__ int s_tix[WT][4];         // col2im: per input-window pixel, its T entries (TZ: none)
    __shared__ WinEnt s_ent[64];         // the window's rows (at most one per objective channel)
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
    // The prologue's loads are issued in dependent levels, each level's loads in flight
    // together: instance and window range -> (entries, relaxation inputs, box, weights) ->
    // the entries' previous bounds.
    const int* wptr = a.win_ptr + (long)ib * (nwin + 1);
    const int e0 = wptr[w];
    const int nrows = min(wptr[w + 1] - e0, 64);
    WinEnt ent{};
    if (t < nrows) ent = a.win_ent[e0 + t];

    // ---- owned window entries (c1 = 4 lk + v, pe = lr): relaxation of ReLU layer 0 and bias
    const int dy = lr / a.ok, dx = lr - dy * a.ok;
    const int Y = Yb + dy, X = Xb + dx;
    const bool pin = lr < P && Y >= 0 && Y < a.Ho && X >= 0 && X < a.Wo;
    const long so0 = (long)in.slot * a.ld_state + Y * a.Wo + X;
    const long po0 = ((long)in.slot * a.n_sets + in.set) * a.ld_param + Y * a.Wo + X;
    float rl[4], ru[4], ral[4], b1v[4];
    int rs[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int c1 = 4 * lk + v;
        rl[v] = ru[v] = ral[v] = 0.f;
        rs[v] = 0;
        if (pin) {
            const long so = so0 + (long)c1 * HoWo;
            rl[v] = a.l[so];
            ru[v] = a.u[so];
            rs[v] = (int)a.S[so];
            ral[v] = a.alpha[po0 + (long)c1 * HoWo];
        }
        b1v[v] = a.b1[c1];
    }
    // ---- owned input-window pixels q = lane + 64 i: (ciq, Ib + qy, Jb + qx), box and A_s
    float lo_q[4], hi_q[4], as_q[4];
    bool qv[4];
    const long qo = (long)a.qid[in.slot] * a.d0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = lane + 64 * i;
        const int ciq = q / IH2, rq = q - ciq * IH2, qy = rq / IH, qx = rq - qy * IH;
        const int py = Ib + qy, px = Jb + qx;
        qv[i] = q < NPIX && py >= 0 && py < a.Hi && px >= 0 && px < a.Wi;
        lo_q[i] = hi_q[i] = as_q[i] = 0.f;
        if (qv[i]) {
            const long o = (long)ciq * HiWi + py * a.Wi + px;
            lo_q[i] = a.lo[qo + o];
            hi_q[i] = a.hi[qo + o];
            as_q[i] = a.asplit[(long)ib * a.d0 + o];
        }
    }
    // col2im table (pixel t): T entries [pos][tap] of the taps that reach it, in (ky, kx) order
    {
        const int q = t;
        const int ciq = q / IH2, rq = q - ciq * IH2, qy = rq / IH, qx = rq - qy * IH;
        int u = 0;
        if (q < NPIX)
            for (int ky = qy % a.s; ky < a.k; ky += a.s) {
                const int pdy = (qy - ky) / a.s;
                if (qy < ky || pdy >= a.ok) continue;
                for (int kx = qx % a.s; kx < a.k; kx += a.s) {
                    const int pdx = (qx - kx) / a.s;
                    if (qx < kx || pdx >= a.ok) continue;
                    if (u < 4) s_tix[q][u++] = (pdy * a.ok + pdx) * 32 + (ciq * a.k + ky) * a.k + kx;
                }
            }
        for (; u < 4; ++u) s_tix[q][u] = TZ;
        if (t < NW) s_T[t][TZ] = 0.f;
    }
    // ---- MFMA operands held in registers: transposed B[k = c1 = 4 lk + ks][n = tap = 16 nt + lr],
    // adjoint A[m = c1 = lr][k = tap = 4 ks + lk] and its B operand's x* index (pos = lr)
    float bT[NT][4], aW[4 * NT];
    int xi[4 * NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int tap = nt * 16 + lr;
            bT[nt][ks] = tap < N ? a.W1[(4 * lk + ks) * N + tap] : 0.f;
        }
#pragma unroll
    for (int ks = 0; ks < 4 * NT; ++ks) {
        const int tap = 4 * ks + lk;
        aW[ks] = tap < N ? a.W1[lr * N + tap] : 0.f;
        int idx = -1;
        if (tap < N && lr < P) {
            const int ci = tap / kk, rr = tap - ci * kk, ky = rr / a.k, kx = rr - ky * a.k;
            idx = (ci * IH + a.s * dy + ky) * IH + a.s * dx + kx;
        }
        xi[ks] = idx;
    }
    if (t < nrows) {
        // the objective neuron's bound before this evaluation (mode 0); each (slot, neuron) of
        // the objective layer has exactly one row in a pass
        if (a.mode == 0) {
            const long o = (long)in.slot * a.ld_state + a.state_off_obj + ent.j;
            const float* src = ent.r >= 0 ? a.lw : a.uw;
            ent.old = src[o];
        }
        s_ent[t] = ent;
    }
    // objective filter entries of the wavefront's first row, loaded ahead like the later ones
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    float wn[4];
    {
        const int co2 = wv < nrows ? a.win_ent[e0 + wv].j / nwin : 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) wn[v] = (wv < nrows && pin) ? a.Wobj[(long)co2 * E + (4 * lk + v) * P + lr] : 0.f;
    }
    float rdp[4], rdn[4], rbn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float l = rl[v], u = ru[v];
        const int sj = rs[v];
        float dp = 0.f, dn = 0.f, bn = 0.f;
        if (!pin || sj == 1) {
        } else if (sj == -1 || l >= 0.f) {
            dp = dn = 1.f;
        } else if (u <= 0.f) {
        } else {
            dp = ral[v];
            const float wd = u - l;
            dn = u / wd;
            bn = -(u * l) / wd;
        }
        rdp[v] = dp;
        rdn[v] = dn;
        rbn[v] = bn;
    }
    // split terms outside the window: the instance totals minus the window's share
    float Lw = 0.f;   // every wavefront owns the same pixels: each sums them itself
    {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (qv[i]) {
                Lw += fminf(as_q[i] * lo_q[i], as_q[i] * hi_q[i]);
            }
    }
    Lw = wave_sum(Lw);
    const float* sc = a.scal + (long)ib * 4;
    const float L_out = sc[0] - Lw, c_split = sc[2];
    __syncthreads();   // s_tix and s_ent complete

    float da[4] = {0.f, 0.f, 0.f, 0.f}, xs[4] = {0.f, 0.f, 0.f, 0.f};
    float* sT = s_T[wave];
    float* sx = s_x[wave];
    for (int ri = wave; ri < nrows; ri += NW) {
        const WinEnt en = s_ent[ri];
        const bool upos = en.r >= 0;   // lower-bound row (+e_j); upper rows store ~r
        const int r = upos ? en.r : ~en.r;
        const float sgn = upos ? 1.f : -1.f;
        float ap[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) ap[v] = sgn * wn[v];
        if (ri + NW < nrows) {
            const int co2 = s_ent[ri + NW].j / nwin;
#pragma unroll
            for (int v = 0; v < 4; ++v) wn[v] = pin ? a.Wobj[(long)co2 * E + (4 * lk + v) * P + lr] : 0.f;
        }
        // fold of ReLU layer 0 on the window (Eq. 5); S beta is in the instance terms
        float ah[4], ce = 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const bool neg = ap[v] < 0.f;
            ah[v] = ap[v] * (neg ? rdn[v] : rdp[v]);
            ce += (neg ? ap[v] * rbn[v] : 0.f) + ah[v] * b1v[v];
        }
        // transposed first convolution on the window: T[pos][tap] = sum_c1 ahat[c1][pos] W1[c1][tap];
        // lane holds T[pos = 4 lk + v][tap = 16 nt + lr]
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[ks], bT[nt][ks], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) sT[(4 * lk + v) * 32 + nt * 16 + lr] = acc[v];
        }
        wave_sync();
        // col2im onto the input window plus A_s, then concretisation over the box (Eq. 6)
        float lbp = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = lane + 64 * i;
            float xq = 0.f;
            if (qv[i]) {
                float acc = as_q[i];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc += sT[s_tix[q][u]];
                lbp += fminf(acc * lo_q[i], acc * hi_q[i]);
                xq = acc < 0.f ? hi_q[i] : lo_q[i];
            }
            sx[q] = xq;
            xs[i] += xq;
        }
        lbp = wave_sum(lbp);
        ce = wave_sum(ce);
        if (lane == 0) {
            const float cpt = (ce + c_split) + en.cb;
            float lb = (L_out + lbp) + cpt;   // intermediate rows: no rounding margin
            if (!(lb == lb) || isinf(lb)) lb = -INFINITY;
            if (a.mode == 0) {
                const long e = (long)in.slot * a.ld_state + a.state_off_obj + en.j;
                if (upos)
                    a.lw[e] = fmaxf(en.old, lb);
                else
                    a.uw[e] = fminf(en.old, isinf(lb) ? INFINITY : -lb);
            } else {
                a.lb_out[r] = lb;
            }
        }
        if (a.adjoint) {
            // ghat^T on the window: W1 im2col(x*)^T; lane holds ghat[c1 = 4 lk + v][pos = lr]
            wave_sync();
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4 * NT; ++ks) {
                if (4 * ks >= N) break;
                const float xv = xi[ks] >= 0 ? sx[xi[ks]] : 0.f;
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aW[ks], xv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float gh = acc[v] + b1v[v];
                if (rbn[v] > 0.f && !(ap[v] < 0.f)) da[v] += ap[v] * gh;
            }
        }
        vmem_drain();   // the next row's filter entries have arrived; nothing left in flight
    }
    // merge the wavefronts' sums in a fixed order
    __syncthreads();
    float* m_a = &s_T[0][0];   // [NW][256] alpha partials by entry
    float* m_x = &s_x[0][0];   // [NW][256] x* sums by pixel
#pragma unroll
    for (int v = 0; v < 4; ++v) m_a[wave * 256 + (4 * lk + v) * 16 + lr] = da[v];
#pragma unroll
    for (int i = 0; i < 4; ++i) m_x[wave * 256 + lane + 64 * i] = xs[i];
    __syncthreads();
    if (!a.adjoint) return;
    const long blk = (long)ib * nwin + w;
    if (t < E) {
        const int c1 = t / P, pe = t - c1 * P;
        const int k2 = c1 * 16 + pe;
        a.part_a[blk * E + t] = ((m_a[k2] + m_a[256 + k2]) + m_a[512 + k2]) + m_a[768 + k2];
    }
    if (t < NPIX) {
        const float xq = ((m_x[t] + m_x[256 + t]) + m_x[512 + t]) + m_x[768 + t];
        const int ciq = t / IH2, rq = t - ciq * IH2, qy = rq / IH, qx = rq - qy * IH;
        const int py = Ib + qy, px = Jb + qx;
        const bool v = py >= 0 && py < a.Hi && px >= 0 && px < a.Wi;
        float xb = 0.f;
        if (v) {
            const long o = (long)ciq * HiWi + py * a.Wi + px;
            xb = a.asplit[(long)ib * a.d0 + o] < 0.f ? a.hi[qo + o] : a.lo[qo + o];
        }
        a.part_x[blk * NPIX + t] = v ? xq - (float)nrows * xb : 0.f;
    }
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
    // at most 2 x 2 first-layer taps reach an input pixel (col2im table of 4 entries)
    return C1 == 16 && ok * ok <= 16 && Ci * IH * IH <= WT && Ci * k * k <= 32 && oCo <= 64 && (k + s - 1) / s <= 2 &&
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
    const int nwin = a.oHo * a.oWo;
    MNB_CHECK(nwin <= 64 && a.win_ptr && a.win_ent, MNB_EDEVICE, "window bottom kernel: row lists");
    const dim3 grid(nwin, n_inst);
    if (N <= 16)
        hipLaunchKernelGGL(k_bottom_win<1>, grid, dim3(WT), 0, st, a);
    else
        hipLaunchKernelGGL(k_bottom_win<2>, grid, dim3(WT), 0, st, a);
    MNB_HIP(hipGetLastError());
}

void launch_win_rows(const WinArgs& a, int n_inst, hipStream_t st) {
    const int nwin = a.oHo * a.oWo;
    if (n_inst <= 0) return;
    MNB_CHECK(nwin <= 64 && a.win_ptr && a.win_ent, MNB_EDEVICE, "window row lists: shape");
    hipLaunchKernelGGL(k_win_rows, dim3(n_inst), dim3(WT), (size_t)a.oCo * nwin * sizeof(int), st, a);
    MNB_HIP(hipGetLastError());
}

void launch_bottom_win_reduce(const WinArgs& a, int n_inst, hipStream_t st) {
    if (!a.adjoint || n_inst <= 0) return;
    const int N = a.Ci * a.k * a.k;
    hipLaunchKernelGGL(k_win_reduce, dim3(n_inst), dim3(WT), (a.d0 + a.C1 * N) * sizeof(float), st, a);
    MNB_HIP(hipGetLastError());
}

}  // namespace mnb
