// Receptive-field ("patch") rows of intermediate-bound passes.
//
// An intermediate-bound row +-e_j on the output of a convolution (the rows that recompute the
// bounds of a ReLU layer after a split, Section 3.2) reaches, through that convolution and every
// convolution below it (Eq. 2), only the input window that neuron j sees.  The ReLU fold (Eq. 5)
// however adds the split and constraint terms S beta + Phat^T gamma of the row's parameter set to
// every row of the set, inside its window or not, and these terms spread through the layers
// below.  The pass therefore splits each row into the set's shared row (the back-substitution of
// the zero objective: the part every row of the set has in common, one whole-layer row per set)
// and the row's deviation from it.  By induction over the layers the deviation is zero outside
// the row's window: outside it a row's coefficient equals the shared row's, so its relaxation
// (which depends only on the sign of a') and hence its folded value agree too, and a transposed
// convolution carries the window of one node into the window of the next.  The deviation rows
// are stored as windows [C][P][P] with origin (y_j S - Q, x_j S - Q) for the objective position
// (y_j, x_j); their transposed convolutions are plain convolutions of the window (no padding).
// The fold and the concretisation (Eq. 6) add back the shared row where the relaxation needs
// the full coefficient.  The adjoint runs on whole rows rebuilt from the two parts.
#include "kernels.h"

#include <algorithm>

namespace mnb {

__device__ __forceinline__ void patch_origin(const PatchGeom& g, int j, int& oy, int& ox) {
    const int pos = j % g.HWobj;
    const int yo = pos / g.Wobj, xo = pos - yo * g.Wobj;
    oy = yo * g.S - g.Q;
    ox = xo * g.S - g.Q;
}

// ------------------------------------------------------------------ row initialisation
// Rows +-e_j on the output of a convolution, j = (co, position): the window on the
// convolution's input is sign * W[co] (all Ci k k taps), the row constant sign * bias[j].
// (The shared row is zero there.)
__global__ __launch_bounds__(256) void k_init_conv_patch(const RowDesc* rows, int M, const float* W,
                                                         const float* bias_eff, int per_co, int HWobj, float* A,
                                                         float* c, int nblk) {
    const long bid = blockIdx.x;
    const int r = (int)(bid / nblk), eb = (int)(bid - (long)r * nblk);
    if (r >= M) return;
    const RowDesc rd = rows[r];
    const float sg = (float)rd.sign;
    const int co = rd.j / HWobj;
    const int e = eb * 256 + threadIdx.x;
    if (e < per_co) A[(long)r * per_co + e] = sg * W[(long)co * per_co + e];
    if (eb == 0 && threadIdx.x == 0) c[r] = sg * bias_eff[rd.j];
}

void launch_init_conv_patch(const RowDesc* rows, int M, const float* W, const float* bias_eff, int per_co,
                            int HWobj, float* A, float* c, hipStream_t st) {
    if (M <= 0) return;
    const int nblk = cdiv(per_co, 256);
    hipLaunchKernelGGL(k_init_conv_patch, dim3((unsigned)((long)M * nblk)), dim3(256), 0, st, rows, M, W, bias_eff,
                       per_co, HWobj, A, c, nblk);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ fold (Eq. 5) of deviation windows
// One workgroup per (row, 256 window entries).  With U' the shared row's a' and d the row's
// deviation, the row's a' is U' + d; the deviation of ahat is (U' + d) D(U' + d) - U' D(U') (the
// set's S beta + Phat^T gamma cancel), the deviation of the row constant
// (U' + d) b(U' + d) - U' b(U') + dev(ahat) . bias; gamma . p is in the shared row's constant.
// Where both sides select the same slope the deviation is formed as d D (no cancellation).
__global__ __launch_bounds__(256) void k_relu_fold_patch(FoldArgs a, PatchGeom g, const RowDesc* rows, int inst_base,
                                                         int nblk) {
    const long bid = blockIdx.x;
    const int r = (int)(bid / nblk), eb = (int)(bid - (long)r * nblk);
    const RowDesc rd = rows[r];
    const int li = rd.inst - inst_base;
    const InstDesc in = a.inst[li];
    const int width = g.C * g.P * g.P;
    const int e = eb * 256 + threadIdx.x;
    const bool ok = e < width;
    int oy, ox;
    patch_origin(g, rd.j, oy, ox);
    const int PP = g.P * g.P;
    const int c = ok ? e / PP : 0;
    const int q = ok ? e - c * PP : 0;
    const int Y = oy + q / g.P, X = ox + q % g.P;
    const bool inside = ok && Y >= 0 && Y < g.H && X >= 0 && X < g.W;
    const int n = inside ? (c * g.H + Y) * g.W + X : 0;
    (void)in;
    float contrib = 0.f;
    const long idx = (long)r * width + e;
    const float dv = ok ? a.A[idx] : 0.f;
    if (inside) {
        const float4 t = a.rt_in[(long)li * a.d + n];   // {D(a' >= 0), D(a' < 0), b, U'}
        const float U = t.w;
        const float ap = U + dv;
        const bool neg = ap < 0.f, uneg = U < 0.f;
        float dh, dc;
        if (neg == uneg) {
            const float D = neg ? t.y : t.x;
            dh = dv * D;
            dc = neg ? dv * t.z : 0.f;
        } else {
            dh = ap * (neg ? t.y : t.x) - U * (uneg ? t.y : t.x);
            dc = (neg ? ap * t.z : 0.f) - (uneg ? U * t.z : 0.f);
        }
        a.A[idx] = dh;
        if (a.Ap) a.Ap[idx] = dv;
        contrib = dc + dh * a.bias[n];
    } else if (ok) {
        a.A[idx] = 0.f;
        if (a.Ap) a.Ap[idx] = 0.f;
    }
    contrib = wave_sum(contrib);
    if ((threadIdx.x & 63) == 0) a.cpart[(long)r * a.ldcp + a.col_off + eb * 4 + (threadIdx.x >> 6)] = contrib;
}

// The same fold with four consecutive window entries per lane (windows of a multiple of 4 entries):
// one wavefront per 256 entries, 16-byte loads and stores, index arithmetic by float reciprocals
// (exact here: entries and window sides are far below 2^22), and the partial constants still one
// per 64 entries (the sum over each 16-lane row).
__global__ __launch_bounds__(256) void k_relu_fold_patch4(FoldArgs a, PatchGeom g, const RowDesc* rows,
                                                          int inst_base, int nblk, float inv_pp, float inv_p) {
    const long bid = blockIdx.x;
    const int r = (int)(bid / nblk), eb = (int)(bid - (long)r * nblk);
    const int lane = threadIdx.x & 63, chunk = eb * 4 + (threadIdx.x >> 6);
    const int width = g.C * g.P * g.P;
    if (chunk * 256 >= width) return;   // wavefront-uniform
    const RowDesc rd = rows[r];
    const int li = rd.inst - inst_base;
    int oy, ox;
    patch_origin(g, rd.j, oy, ox);
    const int PP = g.P * g.P;
    const int e0 = chunk * 256 + 4 * lane;
    const bool ok = e0 < width;
    const long idx = (long)r * width + (ok ? e0 : 0);
    const float4 dv4 = ok ? *reinterpret_cast<const float4*>(a.A + idx) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float dvs[4] = {dv4.x, dv4.y, dv4.z, dv4.w};
    float dh[4], contrib = 0.f;
    bool ins[4];
    int nn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = e0 + k;
        const int c = (int)(((float)e + 0.5f) * inv_pp);
        const int q = e - c * PP;
        const int qy = (int)(((float)q + 0.5f) * inv_p);
        const int Y = oy + qy, X = ox + q - qy * g.P;
        ins[k] = ok && Y >= 0 && Y < g.H && X >= 0 && X < g.W;
        nn[k] = ins[k] ? (c * g.H + Y) * g.W + X : 0;
    }
    float4 tt[4];
    float bb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        tt[k] = a.rt_in[(long)li * a.d + nn[k]];   // {D(a' >= 0), D(a' < 0), b, U'}
        bb[k] = a.bias[nn[k]];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dh[k] = 0.f;
        if (!ins[k]) continue;
        const float4 t = tt[k];
        const float U = t.w, d = dvs[k];
        const float ap = U + d;
        const bool neg = ap < 0.f, uneg = U < 0.f;
        float dc;
        if (neg == uneg) {
            const float D = neg ? t.y : t.x;
            dh[k] = d * D;
            dc = neg ? d * t.z : 0.f;
        } else {
            dh[k] = ap * (neg ? t.y : t.x) - U * (uneg ? t.y : t.x);
            dc = (neg ? ap * t.z : 0.f) - (uneg ? U * t.z : 0.f);
        }
        contrib += dc + dh[k] * bb[k];
    }
    if (ok) {
        *reinterpret_cast<float4*>(a.A + idx) = make_float4(dh[0], dh[1], dh[2], dh[3]);
        if (a.Ap)
            *reinterpret_cast<float4*>(a.Ap + idx) = make_float4(ins[0] ? dvs[0] : 0.f, ins[1] ? dvs[1] : 0.f,
                                                                 ins[2] ? dvs[2] : 0.f, ins[3] ? dvs[3] : 0.f);
    }
    contrib = row16_sum(contrib);
    if ((lane & 15) == 15) a.cpart[(long)r * a.ldcp + a.col_off + chunk * 4 + (lane >> 4)] = contrib;
}

void launch_relu_fold_patch(const FoldArgs& a, const PatchGeom& g, const RowDesc* rows, int inst_base,
                            hipStream_t st) {
    if (a.M <= 0) return;
    const int width = g.C * g.P * g.P;
    if (width % 4 == 0 && ((uintptr_t)a.A & 15) == 0 && (!a.Ap || ((uintptr_t)a.Ap & 15) == 0)) {
        const int nblk = cdiv(width, 1024);
        hipLaunchKernelGGL(k_relu_fold_patch4, dim3((unsigned)((long)a.M * nblk)), dim3(256), 0, st, a, g, rows,
                           inst_base, nblk, 1.f / (float)(g.P * g.P), 1.f / (float)g.P);
    } else {
        const int nblk = cdiv(width, 256);
        hipLaunchKernelGGL(k_relu_fold_patch, dim3((unsigned)((long)a.M * nblk)), dim3(256), 0, st, a, g, rows,
                           inst_base, nblk);
    }
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ whole rows from the two parts
// out[r][n] = shared[instance of r][n] (+ the window entry of row r at n, if win and n lies in
// the window).  One workgroup per (row, 256 neurons).
__global__ __launch_bounds__(256) void k_patch_expand(const float* shared, const float* win, const RowDesc* rows,
                                                      int inst_base, PatchGeom g, float* out, int nblk) {
    const long bid = blockIdx.x;
    const int r = (int)(bid / nblk), b = (int)(bid - (long)r * nblk);
    const int d = g.C * g.H * g.W;
    const int n = b * 256 + threadIdx.x;
    if (n >= d) return;
    const RowDesc rd = rows[r];
    const int li = rd.inst - inst_base;
    float v = shared[(long)li * d + n];
    if (win) {
        int oy, ox;
        patch_origin(g, rd.j, oy, ox);
        const int c = n / (g.H * g.W), rem = n - c * g.H * g.W;
        const int dy = rem / g.W - oy, dx = rem % g.W - ox;
        if (dy >= 0 && dy < g.P && dx >= 0 && dx < g.P)
            v += win[(long)r * g.C * g.P * g.P + (c * g.P + dy) * g.P + dx];
    }
    out[(long)r * d + n] = v;
}

void launch_patch_expand(const float* shared, const float* win, const RowDesc* rows, int M, int inst_base,
                         const PatchGeom& g, float* out, hipStream_t st) {
    if (M <= 0) return;
    const int nblk = cdiv((long)g.C * g.H * g.W, 256);
    hipLaunchKernelGGL(k_patch_expand, dim3((unsigned)((long)M * nblk)), dim3(256), 0, st, shared, win, rows,
                       inst_base, g, out, nblk);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ adjoint on forward cones
// Shared rows' relaxation of forward values: g = D(U') ghat + b(U') per (instance, neuron).
__global__ __launch_bounds__(256) void k_relax_shared(RelaxArgs a, const float* ush, const float* ghs, float* gs) {
    const int li = blockIdx.y;
    const InstDesc in = a.inst[li];
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= a.d) return;
    const long so = (long)in.slot * a.ld_state + n;
    const long po = ((long)in.slot * a.n_sets + in.set) * a.ld_param + n;
    const NeuronRelax nr = neuron_relax(a.l[so], a.u[so], (int)a.S[so], a.alpha[po]);
    const long i = (long)li * a.d + n;
    const bool un = ush[i] < 0.f;
    gs[i] = (un ? nr.dneg : nr.dpos) * ghs[i] + (un ? nr.bneg : 0.f);
}

void launch_relax_shared(const RelaxArgs& a, const float* ush, const float* ghs, float* gs, hipStream_t st) {
    if (a.n_inst <= 0) return;
    hipLaunchKernelGGL(k_relax_shared, dim3(cdiv(a.d, 256), a.n_inst), dim3(256), 0, st, a, ush, ghs, gs);
    MNB_HIP(hipGetLastError());
}

// The relaxation step of the adjoint (g = D ghat + b, with the parameter-gradient sums of every
// instance, as k_relu_relax) for rows held as deviations from their instance's shared row: Gd
// holds each row's forward deviation on its cone, apw its a' deviation on its window.  One
// thread per (instance, CG channels, node position, slice of kRowSlice rows); it walks the
// slice's rows in order (their cone and window origins staged in LDS), takes the rows whose cone
// holds its position and, for each of its channels, writes their new deviation; every other row
// equals the shared row there, whose terms enter the slice's sums once per such row.  A
// wavefront first tests, with scalar instructions, whether a row's cone reaches the band of node
// rows its positions lie in, and skips it otherwise.  Cone entries outside the node are left to
// the convolution that wrote the cone (or k_cone_zero).
template <int CG>
__global__ __launch_bounds__(256) void k_relax_cone(RelaxArgs a, PatchGeom gw, PatchGeom gc, const RowDesc* rows,
                                                    const float* ush, const float* ghs, const float* apw, float* Gd) {
    const int li = blockIdx.y;
    InstDesc in = a.inst[li];
    // this workgroup's slice of the instance's rows
    const int z = blockIdx.z;
    const int nrows = in.r1 - in.r0;
    if (z * kRowSlice >= nrows) return;
    in.r0 += z * kRowSlice;
    in.r1 = min(in.r1, in.r0 + kRowSlice);
    const int HW = gc.H * gc.W;
    const int ngrp = gc.C / CG;
    const int total = ngrp * HW;
    const int t = blockIdx.x * 256 + threadIdx.x;
    const bool act = t < total;
    const int tt = act ? t : 0;
    const int cg = tt / HW;
    const int rem = tt - cg * HW;
    const int c0 = cg * CG;
    const int Y = rem / gc.W, X = rem - Y * gc.W;
    const int n0 = (c0 * gc.H + Y) * gc.W + X;
    // node rows of this wavefront's positions (all rows if it spans two channel groups)
    const int tw0 = __builtin_amdgcn_readfirstlane(blockIdx.x * 256 + (threadIdx.x & ~63));
    const int tw1 = min(tw0 + 63, total - 1);
    const int g0 = tw0 / HW, g1 = tw1 / HW;
    const int Ya = g0 == g1 ? (tw0 - g0 * HW) / gc.W : 0;
    const int Yb = g0 == g1 ? (tw1 - g1 * HW) / gc.W : gc.H - 1;
    NeuronRelax nr[CG];
    float U[CG], Gh[CG], Gs[CG], da[CG], sh[CG], sg[CG];
    bool un[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q) {
        const int n = n0 + q * HW;
        const long so = (long)in.slot * a.ld_state + n;
        const long po = ((long)in.slot * a.n_sets + in.set) * a.ld_param + n;
        nr[q] = neuron_relax(a.l[so], a.u[so], (int)a.S[so], a.alpha[po]);
        U[q] = ush[(long)li * a.d + n];
        Gh[q] = ghs[(long)li * a.d + n];
        un[q] = U[q] < 0.f;
        Gs[q] = (un[q] ? nr[q].dneg : nr[q].dpos) * Gh[q] + (un[q] ? nr[q].bneg : 0.f);
        da[q] = sh[q] = sg[q] = 0.f;
    }
    const int Pc = gc.P, Pw = gw.P;
    const int cw = gc.C * Pc * Pc, ww = gw.C * Pw * Pw;
    const long coff = (long)c0 * Pc * Pc, woff = (long)c0 * Pw * Pw;
    int cnt = 0;
    __shared__ int4 org[kRowSlice];
    const int nrow = in.r1 - in.r0;
    if ((int)threadIdx.x < nrow) {
        const int pos = rows[in.r0 + threadIdx.x].j % gc.HWobj;
        const int yo = pos / gc.Wobj, xo = pos - yo * gc.Wobj;
        org[threadIdx.x] = make_int4(yo * gc.S - gc.Q, xo * gc.S - gc.Q, yo * gw.S - gw.Q, xo * gw.S - gw.Q);
    }
    __syncthreads();
    if (!act) return;
    // RU rows at a time: the covered rows' loads of a group are in flight together
    constexpr int RU = 4;
    for (int k0 = 0; k0 < nrow; k0 += RU) {
        bool cov[RU], inw[RU], band[RU];
        float* ge[RU];
        const float* we[RU];
        bool anyband = false;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int k = k0 + u < nrow ? k0 + u : nrow - 1;
            const int oy = __builtin_amdgcn_readfirstlane(org[k].x);
            band[u] = k0 + u < nrow && oy <= Yb && oy + Pc > Ya;   // wavefront-uniform
            anyband |= band[u];
        }
        if (!anyband) continue;
        bool any = false;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            cov[u] = false;
            inw[u] = false;
            ge[u] = Gd;
            we[u] = apw;
            if (!band[u]) continue;
            const int4 o = org[k0 + u];
            const int dy = Y - o.x, dx = X - o.y, wy = Y - o.z, wx = X - o.w;
            cov[u] = (unsigned)dy < (unsigned)Pc && (unsigned)dx < (unsigned)Pc;
            inw[u] = (unsigned)wy < (unsigned)Pw && (unsigned)wx < (unsigned)Pw;
            ge[u] = Gd + (long)(in.r0 + k0 + u) * cw + coff + (cov[u] ? dy * Pc + dx : 0);
            we[u] = apw + (long)(in.r0 + k0 + u) * ww + woff + (inw[u] ? wy * Pw + wx : 0);
            any |= cov[u];
        }
        if (!any) continue;
        float dgh[RU][CG], dv[RU][CG];
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int q = 0; q < CG; ++q) {
                dgh[u][q] = cov[u] ? ge[u][q * Pc * Pc] : 0.f;
                dv[u][q] = (cov[u] && inw[u]) ? we[u][q * Pw * Pw] : 0.f;
            }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            if (!cov[u]) continue;
#pragma unroll
            for (int q = 0; q < CG; ++q) {
                const float gh = Gh[q] + dgh[u][q];
                const float ap = U[q] + dv[u][q];
                const bool neg = ap < 0.f;
                const float D = neg ? nr[q].dneg : nr[q].dpos;
                const float g = D * gh + (neg ? nr[q].bneg : 0.f);
                ge[u][q * Pc * Pc] = neg == un[q] ? D * dgh[u][q] : g - Gs[q];
                if (nr[q].unstable && !neg) da[q] += ap * gh;
                sh[q] += gh;
                sg[q] += g;
            }
            ++cnt;
        }
    }
    // rows of the slice whose cone misses this position carry the shared row's terms
    const float rest = (float)(nrow - cnt);
    float* pz = a.part + (long)(a.zoff[li] + z) * 3 * a.d;
#pragma unroll
    for (int q = 0; q < CG; ++q) {
        const int n = n0 + q * HW;
        if (nr[q].unstable && !un[q]) da[q] += rest * (U[q] * Gh[q]);
        sh[q] += rest * Gh[q];
        sg[q] += rest * Gs[q];
        pz[n] = da[q];
        pz[a.d + n] = sh[q];
        pz[2 * a.d + n] = sg[q];
    }
}

// Cone entries outside the node hold 0 (the next convolution reads them as padding): workgroups
// stride over the rows, their lanes over a row's cone positions (consecutive lanes, consecutive
// entries), each position outside the node zeroed in every channel.
__global__ __launch_bounds__(256) void k_cone_zero(PatchGeom gc, const RowDesc* rows, int M, float* Gd, float inv_p) {
    const int Pc = gc.P, PP = Pc * Pc;
    for (long r = blockIdx.x; r < M; r += gridDim.x) {
        int oy, ox;
        patch_origin(gc, rows[r].j, oy, ox);
        // a cone inside the node has nothing to clear
        if (oy >= 0 && ox >= 0 && oy + Pc <= gc.H && ox + Pc <= gc.W) continue;
        float* base = Gd + r * gc.C * PP;
        for (int q = threadIdx.x; q < PP; q += 256) {
            const int dy = (int)(((float)q + 0.5f) * inv_p), dx = q - dy * Pc;
            const int Y = oy + dy, X = ox + dx;
            if (Y >= 0 && Y < gc.H && X >= 0 && X < gc.W) continue;
            for (int c = 0; c < gc.C; ++c) base[(long)c * PP + q] = 0.f;
        }
    }
}

void launch_cone_zero(const PatchGeom& gc, const RowDesc* rows, int M, float* Gd, hipStream_t st) {
    if (M <= 0) return;
    hipLaunchKernelGGL(k_cone_zero, dim3((unsigned)std::min(M, 2048)), dim3(256), 0, st, gc, rows, M, Gd,
                       1.f / (float)gc.P);
    MNB_HIP(hipGetLastError());
}

void launch_relax_cone(const RelaxArgs& a, const PatchGeom& gw, const PatchGeom& gc, const RowDesc* rows,
                       const float* ush, const float* ghs, const float* apw, float* Gd, hipStream_t st) {
    if (a.n_inst <= 0) return;
    const int HW = gc.H * gc.W;
    if (a.n_slices <= 0) {
        // no rows: the sums below are zero
    } else if (gc.C % 4 == 0) {
        dim3 grid(cdiv((long)(gc.C / 4) * HW, 256), a.n_inst, a.n_slices);
        hipLaunchKernelGGL(k_relax_cone<4>, grid, dim3(256), 0, st, a, gw, gc, rows, ush, ghs, apw, Gd);
    } else {
        dim3 grid(cdiv((long)gc.C * HW, 256), a.n_inst, a.n_slices);
        hipLaunchKernelGGL(k_relax_cone<1>, grid, dim3(256), 0, st, a, gw, gc, rows, ush, ghs, apw, Gd);
    }
    MNB_HIP(hipGetLastError());
    launch_relax_sum(a, st);
}

}  // namespace mnb
