// Memory-bound kernels of back-substitution: ReLU fold (Eq. 5), its adjoint,
// concretisation over the input box (Eq. 6), row initialisation, interval
// propagation, projected Adam, MNC projections, branching score and splits.
//
// Layout: a pass holds M coefficient rows [M, d] (row-major, rows of one
// instance = (subproblem, parameter set) contiguous).  Per-neuron quantities
// shared by an instance's rows are loaded once per thread and the thread walks
// the instance's rows, so every row reduction has a fixed order and a row's
// result does not depend on what else is in the batch.
#include "kernels.h"

#include <algorithm>

namespace mnb {

// ------------------------------------------------------------------ fold (Eq. 5)
__global__ __launch_bounds__(256) void k_relu_fold(FoldArgs a, const float* gp) {
    const InstDesc in = a.inst[blockIdx.y];
    const int j = blockIdx.x * 256 + threadIdx.x;
    const bool ok = j < a.d;
    const int jj = ok ? j : 0;
    const long so = (long)in.slot * a.ld_state + jj;
    const long po = ((long)in.slot * a.n_sets + in.set) * a.ld_param + jj;
    NeuronRelax nr = neuron_relax(a.l[so], a.u[so], (int)a.S[so], a.alpha[po]);
    const int s = (int)a.S[so];
    const float vv = a.v ? a.v[(long)blockIdx.y * a.d + jj] : 0.f;
    const float vh = a.vhat ? a.vhat[(long)blockIdx.y * a.d + jj] : 0.f;
    const float add = (s != 0 ? (float)s * a.beta[po] : 0.f) + vh;
    const float bias = a.bias[jj];
    const float gpv = (gp && blockIdx.x == 0 && threadIdx.x == 0) ? gp[blockIdx.y] : 0.f;
    const int col = a.col_off + blockIdx.x * 4 + (threadIdx.x >> 6);
    // the per-neuron values above complete, in a form the compiler sees: otherwise it waits for
    // them (and, the counter being in order, for every store before) inside the row loop.  The
    // empty asm keeps their loads above the wait.
    asm volatile("" ::: "memory");
    vmem_drain();
    // rows in groups of FR with all of a group's loads in flight together
    constexpr int FR = 8;
    for (int r0 = in.r0; r0 < in.r1; r0 += FR) {
        float av[FR];
        if (a.Wsrc) {
            // the group's row descriptors {b, inst, j, sign} as 16-byte loads, all in flight together
            int4 rdv[FR];
#pragma unroll
            for (int u = 0; u < FR; ++u) rdv[u] = reinterpret_cast<const int4*>(a.rows)[min(r0 + u, in.r1 - 1)];
            float sg[FR];
            int jr[FR];
#pragma unroll
            for (int u = 0; u < FR; ++u) {
                sg[u] = (float)rdv[u].w;
                jr[u] = rdv[u].z;
            }
            // every lane loads (rows past the instance read its last row's filter, lanes past d
            // column 0), so that the loads are in flight together; the value is then selected
#pragma unroll
            for (int u = 0; u < FR; ++u) {
                const float w = a.Wsrc[(long)jr[u] * a.d + jj];
                av[u] = (ok && r0 + u < in.r1) ? sg[u] * w : 0.f;
            }
            if (blockIdx.x == 0 && threadIdx.x < FR && r0 + (int)threadIdx.x < in.r1) {
                const int u = threadIdx.x;
                a.c[r0 + u] = sg[u] * a.bias_obj[jr[u]];
            }
        } else {
#pragma unroll
            for (int u = 0; u < FR; ++u) av[u] = (ok && r0 + u < in.r1) ? a.A[(long)(r0 + u) * a.d + j] : 0.f;
        }
        // the group's values complete before its first store: no later wait (which would also
        // wait for the stores before it) is left pending inside the row steps
        vmem_drain();
#pragma unroll
        for (int u = 0; u < FR; ++u) {
            const int r = r0 + u;
            if (r >= in.r1) break;
            float contrib = 0.f;
            if (ok) {
                const long e = (long)r * a.d + j;
                const float ap = av[u] + vv;
                const bool neg = ap < 0.f;
                const float D = neg ? nr.dneg : nr.dpos;
                const float ah = ap * D + add;
                a.A[e] = ah;
                if (a.Ap) a.Ap[e] = ap;
                if (a.rt_out) a.rt_out[(long)blockIdx.y * a.d + j] = make_float4(nr.dpos, nr.dneg, nr.bneg, ap);
                contrib = (neg ? ap * nr.bneg : 0.f) + ah * bias;
            }
            contrib -= gpv;
            contrib = wave_sum(contrib);
            if ((threadIdx.x & 63) == 0) a.cpart[(long)r * a.ldcp + col] = contrib;
        }
    }
}

void launch_relu_fold(const FoldArgs& a, hipStream_t st, const float* gp) {
    if (a.n_inst <= 0) return;
    dim3 grid(cdiv(a.d, 256), a.n_inst);
    hipLaunchKernelGGL(k_relu_fold, grid, dim3(256), 0, st, a, gp);
    MNB_HIP(hipGetLastError());
}
void launch_relu_fold(const FoldArgs& a, hipStream_t st) { launch_relu_fold(a, st, nullptr); }

// ------------------------------------------------------------------ adjoint relax
// Forward image of the concretisation minimiser through a row's relaxation:
// g = D ghat + b-underline, with the parameter gradients of the row's set
//   d alpha_j = sum_r [unstable, a'_rj >= 0] a'_rj ghat_rj,  d beta_j = S_j sum_r ghat_rj.
__global__ __launch_bounds__(256) void k_relu_relax(RelaxArgs a) {
    const InstDesc in = a.inst[blockIdx.y];
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= a.d) return;
    const long so = (long)in.slot * a.ld_state + j;
    const long po = ((long)in.slot * a.n_sets + in.set) * a.ld_param + j;
    const int s = (int)a.S[so];
    NeuronRelax nr = neuron_relax(a.l[so], a.u[so], s, a.alpha[po]);
    float da = 0.f, sh = 0.f, sg = 0.f;
    // rows in groups of RR with all of a group's loads in flight together; sums in row order
    constexpr int RR = 16;
    for (int r0 = in.r0; r0 < in.r1; r0 += RR) {
        float ghv[RR], apv[RR];
#pragma unroll
        for (int u = 0; u < RR; ++u) {
            const long e = (long)min(r0 + u, in.r1 - 1) * a.d + j;
            ghv[u] = a.G[e];
            apv[u] = a.Ap[e];
        }
#pragma unroll
        for (int u = 0; u < RR; ++u) {
            if (r0 + u >= in.r1) break;
            const float gh = ghv[u], ap = apv[u];
            const bool neg = ap < 0.f;
            const float g = (neg ? nr.dneg : nr.dpos) * gh + (neg ? nr.bneg : 0.f);
            a.G[(long)(r0 + u) * a.d + j] = g;
            if (nr.unstable && !neg) da += ap * gh;
            sh += gh;
            sg += g;
        }
    }
    const long go = (long)blockIdx.y * a.ldg + a.goff + j;
    a.d_alpha[go] = da;
    a.d_beta[go] = (float)s * sh;
    if (a.gsum_hat) a.gsum_hat[(long)blockIdx.y * a.d + j] = sh;
    if (a.gsum_out) a.gsum_out[(long)blockIdx.y * a.d + j] = sg;
}

// Gradient sums of a relaxation run in row slices (the cone relaxation): the slices' partial sums
// of each (instance, neuron) added in slice order.
__global__ __launch_bounds__(256) void k_relax_sum(RelaxArgs a) {
    const int li = blockIdx.y;
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= a.d) return;
    const InstDesc in = a.inst[li];
    float da = 0.f, sh = 0.f, sg = 0.f;
    for (int z = a.zoff[li]; z < a.zoff[li + 1]; ++z) {
        const float* pz = a.part + (long)z * 3 * a.d;
        da += pz[n];
        sh += pz[a.d + n];
        sg += pz[2 * a.d + n];
    }
    const long go = (long)li * a.ldg + a.goff + n;
    a.d_alpha[go] = da;
    a.d_beta[go] = (float)a.S[(long)in.slot * a.ld_state + n] * sh;
    if (a.gsum_hat) a.gsum_hat[(long)li * a.d + n] = sh;
    if (a.gsum_out) a.gsum_out[(long)li * a.d + n] = sg;
}

void launch_relax_sum(const RelaxArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_relax_sum, dim3(cdiv(a.d, 256), a.n_inst), dim3(256), 0, st, a);
    MNB_HIP(hipGetLastError());
}

void launch_relu_relax(const RelaxArgs& a, hipStream_t st) {
    if (a.n_inst <= 0) return;
    dim3 grid(cdiv(a.d, 256), a.n_inst);
    hipLaunchKernelGGL(k_relu_relax, grid, dim3(256), 0, st, a);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ concretisation (Eq. 6)
// lb_r = sum_j min(a_j lo_j, a_j hi_j) + c_r (+ the partial constants of the
// ReLU folds); a spec row's bound is lowered by the rounding margin
// 2^-20 (sum_j |a_j| max(|lo_j|,|hi_j|) + |c_r|), an intermediate row's is not.
// x*_j = hi_j if a_j < 0 else lo_j.
template <bool PATCH>
__global__ __launch_bounds__(256) void k_concretize(ConcArgs a) {
    const int r = blockIdx.x;
    const RowDesc rd = a.rows[r];
    const int slot = a.slots[rd.b];
    const int q = a.qid[slot];
    const float* lo = a.lo + (long)q * a.d0;
    const float* hi = a.hi + (long)q * a.d0;
    float s = 0.f, mag = 0.f;
    if (PATCH) {
        // deviation window of a receptive-field row: the row's coefficient is U + dev, with U the
        // shared row's input coefficients; sum of min(c lo, c hi) - min(U lo, U hi) over the window
        const PatchGeom& g = a.pg;
        const int width = g.C * g.P * g.P;
        const int li = rd.inst - a.inst_base;
        const float* Ush = a.ush0 + (long)li * a.d0;
        const float* A = a.A + (long)r * width;
        const int pos = rd.j % g.HWobj;
        const int oy = (pos / g.Wobj) * g.S - g.Q, ox = (pos % g.Wobj) * g.S - g.Q;
        for (int e = threadIdx.x; e < width; e += 256) {
            const int ch = e / (g.P * g.P), qq = e - ch * g.P * g.P;
            const int Y = oy + qq / g.P, X = ox + qq % g.P;
            if (Y < 0 || Y >= g.H || X < 0 || X >= g.W) {
                if (a.G0 && a.g0_dev) a.G0[(long)r * width + e] = 0.f;
                continue;
            }
            const int j = (ch * g.H + Y) * g.W + X;
            const float dv = A[e], U = Ush[j];
            const float c = U + dv;
            const float l = lo[j], h = hi[j];
            const bool neg = c < 0.f, uneg = U < 0.f;
            if (neg == uneg)
                s += dv * (neg ? h : l);
            else
                s += fminf(c * l, c * h) - fminf(U * l, U * h);
            if (a.G0) {
                if (a.g0_dev)
                    a.G0[(long)r * width + e] = neg == uneg ? 0.f : (neg ? h - l : l - h);
                else
                    a.G0[(long)r * a.d0 + j] = neg ? h : l;
            }
        }
    } else {
        const float* A = a.A + (long)r * a.d0;
        for (int j = threadIdx.x; j < a.d0; j += 256) {
            const float c = A[j];
            const float l = lo[j], h = hi[j];
            s += fminf(c * l, c * h);
            mag += fabsf(c) * fmaxf(fabsf(l), fabsf(h));
            const bool neg = c < 0.f;
            if (a.G0) a.G0[(long)r * a.d0 + j] = neg ? h : l;
            if (a.xbits) a.xbits[(long)r * a.d0 + j] = neg ? 1 : 0;
        }
    }
    __shared__ float red[2][4];
    s = wave_sum(s);
    mag = wave_sum(mag);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s;
        red[1][threadIdx.x >> 6] = mag;
    }
    __syncthreads();
    if (threadIdx.x >= 64) return;
    float c = row_constant(a.c, a.cpart, a.ldcp, a.ncp, r);
    if (PATCH) c += a.lbs[rd.inst - a.inst_base];   // the shared row's bound
    if (threadIdx.x != 0) return;
    const float tot = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3])) + c;
    const float m = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3])) + fabsf(c);
    float lb = tot - m * a.margin;
    if (!(lb == lb) || isinf(lb)) lb = -INFINITY;   // NaN / Inf never gives a positive bound
    if (a.mode == 2) {
        a.lb_out[r] = lb;
    } else if (a.mode == 0) {
        // intermediate bound of neuron rd.j of the objective layer, intersected with the old one
        const long e = (long)slot * a.ld_state + a.state_off + rd.j;
        if (rd.sign > 0) {
            a.l[e] = fmaxf(a.l[e], lb);
        } else {
            const float ub = -lb;
            a.u[e] = fminf(a.u[e], isinf(lb) ? INFINITY : ub);
        }
    } else {
        a.lb_out[r] = lb;
        if (a.best) {
            if (lb > a.best[r]) {
                a.best[r] = lb;
                a.improved[r] = 1;
            } else {
                a.improved[r] = 0;
            }
        }
    }
}

void launch_concretize(const ConcArgs& a, hipStream_t st) {
    if (a.M <= 0) return;
    if (a.pg.P > 0)
        hipLaunchKernelGGL(k_concretize<true>, dim3(a.M), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_concretize<false>, dim3(a.M), dim3(256), 0, st, a);
    MNB_HIP(hipGetLastError());
}

// Copy the x* bits of rows whose best bound improved in the last evaluation.
__global__ void k_keep_best_x(const uint8_t* xbits, uint8_t* best_bits, const uint8_t* improved, int M,
                              int d0) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)M * d0) return;
    int r = (int)(idx / d0);
    if (improved[r]) best_bits[idx] = xbits[idx];
}
void launch_keep_best_x(const uint8_t* xbits, uint8_t* best_bits, const uint8_t* improved, int M,
                        int d0, hipStream_t st) {
    if (M <= 0) return;
    long tot = (long)M * d0;
    hipLaunchKernelGGL(k_keep_best_x, dim3(cdiv(tot, 256)), dim3(256), 0, st, xbits, best_bits, improved,
                       M, d0);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ row initialisation
// Spec rows: coefficients Chat = C W^(L) (the property folded into the last affine layer).
__global__ void k_init_spec(const RowDesc* rows, const int32_t* slots, const int32_t* qid, const float* Chat,
                            const float* chat, int S, int d, float* A, float* c, int r0) {
    const int r = r0 + blockIdx.y;
    const RowDesc rd = rows[r];
    const int q = qid[slots[rd.b]];
    const float* src = Chat + ((long)q * S + rd.j) * d;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < d; j += gridDim.x * 256) A[(long)r * d + j] = src[j];
    if (blockIdx.x == 0 && threadIdx.x == 0) c[r] = chat[(long)q * S + rd.j];
}
void launch_init_spec(const RowDesc* rows, int M, const int32_t* slots, const int32_t* qid,
                      const float* Chat, const float* chat, int S, int d, float* A, float* c,
                      hipStream_t st) {
    if (M <= 0) return;
    for (int r0 = 0; r0 < M; r0 += kMaxGridY) {
        hipLaunchKernelGGL(k_init_spec, dim3(cdiv(d, 256), std::min(M - r0, kMaxGridY)), dim3(256), 0, st, rows,
                           slots, qid, Chat, chat, S, d, A, c, r0);
        MNB_HIP(hipGetLastError());
    }
}

// Intermediate rows +-e_j on the output of an FC node: a = +-W[j, :], c = +-bias[j].
__global__ void k_init_fc(const RowDesc* rows, const float* W, const float* bias_eff, int din, float* A,
                          float* c, int write_c, int r0) {
    const int r = r0 + blockIdx.y;
    const RowDesc rd = rows[r];
    const float sg = (float)rd.sign;
    const float* w = W + (long)rd.j * din;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < din; k += gridDim.x * 256)
        A[(long)r * din + k] = sg * w[k];
    if (write_c && blockIdx.x == 0 && threadIdx.x == 0) c[r] = sg * bias_eff[rd.j];
}
void launch_init_fc(const RowDesc* rows, int M, const float* W, const float* bias_eff, int din, float* A,
                    float* c, bool write_c, hipStream_t st) {
    if (M <= 0) return;
    for (int r0 = 0; r0 < M; r0 += kMaxGridY) {
        hipLaunchKernelGGL(k_init_fc, dim3(cdiv(din, 256), std::min(M - r0, kMaxGridY)), dim3(256), 0, st, rows, W,
                           bias_eff, din, A, c, (int)write_c, r0);
        MNB_HIP(hipGetLastError());
    }
}

// Intermediate rows +-e_j on the output of a conv node (j = (co, y, x)): the
// filter of output channel co placed at its input window.
__global__ void k_init_conv(const RowDesc* rows, const float* W, const float* bias_eff, int Ci, int Hi,
                            int Wi, int Co, int Ho, int Wo, int k, int s, int p, float* A, float* c,
                            int write_c, int r0) {
    const int r = r0 + blockIdx.y;
    const RowDesc rd = rows[r];
    const float sg = (float)rd.sign;
    const int co = rd.j / (Ho * Wo);
    const int pos = rd.j - co * Ho * Wo;
    const int y = pos / Wo, x = pos - y * Wo;
    const int din = Ci * Hi * Wi;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < din; e += gridDim.x * 256) {
        const int ci = e / (Hi * Wi);
        const int q = e - ci * Hi * Wi;
        const int Y = q / Wi, X = q - Y * Wi;
        const int ky = Y - s * y + p, kx = X - s * x + p;
        float v = 0.f;
        if (ky >= 0 && ky < k && kx >= 0 && kx < k) v = sg * W[(((long)co * Ci + ci) * k + ky) * k + kx];
        A[(long)r * din + e] = v;
    }
    if (write_c && blockIdx.x == 0 && threadIdx.x == 0) c[r] = sg * bias_eff[rd.j];
}
void launch_init_conv(const RowDesc* rows, int M, const ConvGeom& g, const float* bias_eff, float* A,
                      float* c, bool write_c, hipStream_t st) {
    if (M <= 0) return;
    const int din = g.Ci * g.Hi * g.Wi;
    for (int r0 = 0; r0 < M; r0 += kMaxGridY) {
        hipLaunchKernelGGL(k_init_conv, dim3(cdiv(din, 256), std::min(M - r0, kMaxGridY)), dim3(256), 0, st, rows,
                           g.W, bias_eff, g.Ci, g.Hi, g.Wi, g.Co, g.Ho, g.Wo, g.k, g.s, g.p, A, c, (int)write_c, r0);
        MNB_HIP(hipGetLastError());
    }
}

// Octahedral rows of multi-neuron constraint generation: row r = 26 g + s carries direction s of
// the 26 in {-1,0,1}^3 \ {0} (lexicographic in (s0, s1, s2), s2 fastest) on the three neurons of
// group g, on the input of a ReLU layer; c_r = s . bias (the input node's bias).  A is zeroed first.
__global__ void k_init_oct(const int32_t* grp, int n_groups, int d, const float* bias, float* A, float* c) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= 26 * n_groups) return;
    const int g = r / 26, s = r - 26 * g;
    const int code = s < 13 ? s : s + 1;   // skip the zero direction, code 13 of the 27
    const int dir[3] = {code / 9 - 1, (code / 3) % 3 - 1, code % 3 - 1};
    float cc = 0.f;
    for (int t = 0; t < 3; ++t) {
        const int j = grp[3 * g + t];
        A[(long)r * d + j] = (float)dir[t];
        cc += (float)dir[t] * bias[j];
    }
    c[r] = cc;
}
void launch_init_oct(const int32_t* grp, int n_groups, int d, const float* bias, float* A, float* c,
                     hipStream_t st) {
    if (n_groups <= 0) return;
    launch_fill(A, (long)26 * n_groups * d, 0.f, st);
    hipLaunchKernelGGL(k_init_oct, dim3(cdiv(26 * n_groups, 128)), dim3(128), 0, st, grp, n_groups, d, bias, A, c);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ interval propagation
// center/radius form of one affine node: c' = W c + b, r' = |W| r.
__global__ void k_ibp_fc(const float* W, const float* b, const float* L, const float* U, float* Lo, float* Uo,
                         int din, int dout) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= dout) return;
    double c = 0.0, rad = 0.0;
    const float* w = W + (long)n * din;
    for (int k = 0; k < din; ++k) {
        double m = 0.5 * ((double)L[k] + (double)U[k]);
        double h = 0.5 * ((double)U[k] - (double)L[k]);
        c += (double)w[k] * m;
        rad += fabs((double)w[k]) * h;
    }
    c += b[n];
    Lo[n] = (float)(c - rad);
    Uo[n] = (float)(c + rad);
}
__global__ void k_ibp_conv(const float* W, const float* b, const float* L, const float* U, float* Lo,
                           float* Uo, int Ci, int Hi, int Wi, int Co, int Ho, int Wo, int k, int s, int p) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= Co * Ho * Wo) return;
    int co = n / (Ho * Wo), pos = n - co * Ho * Wo;
    int y = pos / Wo, x = pos - y * Wo;
    double c = 0.0, rad = 0.0;
    for (int ci = 0; ci < Ci; ++ci)
        for (int ky = 0; ky < k; ++ky)
            for (int kx = 0; kx < k; ++kx) {
                int Y = s * y - p + ky, X = s * x - p + kx;
                if (Y < 0 || Y >= Hi || X < 0 || X >= Wi) continue;
                long e = ((long)ci * Hi + Y) * Wi + X;
                double w = W[(((long)co * Ci + ci) * k + ky) * k + kx];
                c += w * 0.5 * ((double)L[e] + (double)U[e]);
                rad += fabs(w) * 0.5 * ((double)U[e] - (double)L[e]);
            }
    c += b[co];
    Lo[n] = (float)(c - rad);
    Uo[n] = (float)(c + rad);
}
void launch_ibp_fc(const float* W, const float* b, const float* L, const float* U, float* Lo, float* Uo,
                   int din, int dout, hipStream_t st) {
    hipLaunchKernelGGL(k_ibp_fc, dim3(cdiv(dout, 128)), dim3(128), 0, st, W, b, L, U, Lo, Uo, din, dout);
    MNB_HIP(hipGetLastError());
}
void launch_ibp_conv(const ConvGeom& g, const float* L, const float* U, float* Lo, float* Uo,
                     hipStream_t st) {
    int n = g.Co * g.Ho * g.Wo;
    hipLaunchKernelGGL(k_ibp_conv, dim3(cdiv(n, 128)), dim3(128), 0, st, g.W, g.b, L, U, Lo, Uo, g.Ci, g.Hi,
                       g.Wi, g.Co, g.Ho, g.Wo, g.k, g.s, g.p);
    MNB_HIP(hipGetLastError());
}
// relu of an interval, intersected with known input bounds (lk/uk nullable)
__global__ void k_ibp_relu(const float* L, const float* U, const float* lk, const float* uk, float* Lo,
                           float* Uo, int d) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    float l = L[j], u = U[j];
    if (lk) {
        l = fmaxf(l, lk[j]);
        u = fminf(u, uk[j]);
    }
    Lo[j] = fmaxf(l, 0.f);
    Uo[j] = fmaxf(u, 0.f);
}
__global__ void k_add2(const float* a, const float* b, float* o, long n) {
    long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) o[j] = a[j] + b[j];
}
void launch_ibp_relu(const float* L, const float* U, const float* lk, const float* uk, float* Lo,
                     float* Uo, int d, hipStream_t st) {
    hipLaunchKernelGGL(k_ibp_relu, dim3(cdiv(d, 256)), dim3(256), 0, st, L, U, lk, uk, Lo, Uo, d);
    MNB_HIP(hipGetLastError());
}
void launch_add2(const float* a, const float* b, float* o, long n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_add2, dim3(cdiv(n, 256)), dim3(256), 0, st, a, b, o, n);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ projected Adam (ascent)
__global__ void k_adam(AdamArgs a) {
    const InstDesc in = a.inst[blockIdx.y];
    const int k = blockIdx.x * 256 + threadIdx.x;
    const long po = ((long)in.slot * a.n_sets + in.set) * a.ld_param + k;
    const long mo = ((long)in.b * a.n_sets + in.set) * a.ld_param + k;
    const long go = (long)blockIdx.y * a.ldg + k;
    if (k < a.n_ab) {
        // The alpha gradient is zero unless the neuron is unstable and unsplit, the beta
        // gradient zero unless it is split.  A stable neuron stays stable (bounds are only
        // intersected), so its alpha no longer enters any bound; a beta with zero gradient and
        // zero moments does not move.  Only those entries are updated.
        const long so = (long)in.slot * a.ld_state + k;
        // S, l and u in one round trip (no short-circuit), then gradient, moments and parameter
        // in one, before any store
        const int sj = (int)a.S[so];
        const float lj = a.l[so], uj = a.u[so];
        const bool upd_a = (sj == 0) & (lj < 0.f) & (uj > 0.f);
        if (upd_a || sj != 0) {
            const bool al = sj == 0;
            const float g = al ? a.g_alpha[go] : a.g_beta[go];
            const float m0 = al ? a.m_alpha[mo] : a.m_beta[mo];
            const float v0 = al ? a.v_alpha[mo] : a.v_beta[mo];
            const float p0 = al ? a.alpha[po] : a.beta[po];
            const float m = a.b1 * m0 + (1.f - a.b1) * g;
            const float v = a.b2 * v0 + (1.f - a.b2) * g * g;
            const float p = p0 + a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
            if (al) {
                a.m_alpha[mo] = m;
                a.v_alpha[mo] = v;
                a.alpha[po] = fminf(fmaxf(p, 0.f), 1.f);
            } else {
                a.m_beta[mo] = m;
                a.v_beta[mo] = v;
                a.beta[po] = fmaxf(p, 0.f);
            }
        }
    }
    if (a.gamma && k < a.n_gamma) {
        const long pg = ((long)in.slot * a.n_sets + in.set) * a.ld_gamma + k;
        const long mg = ((long)in.b * a.n_sets + in.set) * a.ld_gamma + k;
        const float g = a.g_gamma[(long)blockIdx.y * a.ld_gamma + k];
        const float m = a.b1 * a.m_gamma[mg] + (1.f - a.b1) * g;
        const float v = a.b2 * a.v_gamma[mg] + (1.f - a.b2) * g * g;
        a.m_gamma[mg] = m;
        a.v_gamma[mg] = v;
        const float p = a.gamma[pg] + a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
        a.gamma[pg] = fmaxf(p, 0.f);
    }
}
void launch_adam(const AdamArgs& a, hipStream_t st) {
    if (a.n_inst <= 0) return;
    int n = a.n_ab > a.n_gamma ? a.n_ab : a.n_gamma;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_adam, dim3(cdiv(n, 256), a.n_inst), dim3(256), 0, st, a);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ MNC (Eq. 3) projections
// v_j = sum_e gamma_e P_ej, vhat_j = sum_e gamma_e Phat_ej (column order fixed), gp = gamma . p.
__global__ void k_gamma_proj(GammaArgs a) {
    const InstDesc in = a.inst[blockIdx.y];
    const float* gam = a.gamma + ((long)in.slot * a.n_sets + in.set) * a.ld_gamma + a.goff;
    const int q = a.qid[in.slot];
    const int* cp = a.colptr + (long)q * (a.d + 1);
    const int* ce = a.col_e + (long)q * a.nnz_cap;
    const float* cP = a.col_P + (long)q * a.nnz_cap;
    const float* cH = a.col_Ph + (long)q * a.nnz_cap;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < a.d) {
        float v = 0.f, vh = 0.f;
        for (int t = cp[j]; t < cp[j + 1]; ++t) {
            const float g = gam[ce[t]];
            v += g * cP[t];
            vh += g * cH[t];
        }
        a.v[(long)blockIdx.y * a.d + j] = v;
        a.vhat[(long)blockIdx.y * a.d + j] = vh;
    }
    if (blockIdx.x == 0) {
        // gamma . p over this layer's constraints (one wave, fixed order)
        if (threadIdx.x < 64) {
            const float* p = a.p + (long)q * a.e_cap;
            const int e = a.e_of[q];
            float s = 0.f;
            for (int t = threadIdx.x; t < e; t += 64) s += gam[t] * p[t];
            s = wave_sum(s);
            if (threadIdx.x == 0) a.gp[blockIdx.y] = s;
        }
    }
}
void launch_gamma_proj(const GammaArgs& a, hipStream_t st) {
    if (a.n_inst <= 0) return;
    hipLaunchKernelGGL(k_gamma_proj, dim3(cdiv(a.d, 256), a.n_inst), dim3(256), 0, st, a);
    MNB_HIP(hipGetLastError());
}

// d gamma_e = sum_j P_ej gsum_out_j + Phat_ej gsum_hat_j - nrows p_e  (row order fixed)
__global__ void k_gamma_grad(GammaArgs a, const float* gsum_hat, const float* gsum_out, float* g_gamma,
                             long ldgg) {
    const InstDesc in = a.inst[blockIdx.y];
    const int q = a.qid[in.slot];
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= a.e_cap) return;
    float g = 0.f;
    if (e < a.e_of[q]) {
        const int* rp = a.rowptr + (long)q * (a.e_cap + 1);
        const int* rc = a.row_j + (long)q * a.nnz_cap;
        const float* rP = a.row_P + (long)q * a.nnz_cap;
        const float* rH = a.row_Ph + (long)q * a.nnz_cap;
        const float* so = gsum_out + (long)blockIdx.y * a.d;
        const float* sh = gsum_hat + (long)blockIdx.y * a.d;
        for (int t = rp[e]; t < rp[e + 1]; ++t) g += rP[t] * so[rc[t]] + rH[t] * sh[rc[t]];
        g -= (float)(in.r1 - in.r0) * a.p[(long)q * a.e_cap + e];
    }
    g_gamma[(long)blockIdx.y * ldgg + a.goff + e] = g;
}
void launch_gamma_grad(const GammaArgs& a, const float* gsum_hat, const float* gsum_out, float* g_gamma,
                       long ldgg, hipStream_t st) {
    if (a.n_inst <= 0 || a.e_cap <= 0) return;
    hipLaunchKernelGGL(k_gamma_grad, dim3(cdiv(a.e_cap, 256), a.n_inst), dim3(256), 0, st, a, gsum_hat,
                       gsum_out, g_gamma, ldgg);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ branching score
// score_j = sum over the spec rows of |a'_j| * (-u l/(u-l)) for unstable, unsplit j.
__global__ void k_score(const InstDesc* inst, const float* Ap, int d, const float* l, const float* u,
                        const int8_t* S, long ld_state, int state_off, float* score, long ld_score,
                        int score_off) {
    const InstDesc in = inst[blockIdx.y];
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= d) return;
    const long so = (long)in.slot * ld_state + state_off + j;
    const float lj = l[so], uj = u[so];
    float sc = -INFINITY;
    if (S[so] == 0 && lj < 0.f && uj > 0.f) {
        float acc = 0.f;
        for (int r = in.r0; r < in.r1; ++r) acc += fabsf(Ap[(long)r * d + j]);
        sc = acc * (-(uj * lj) / (uj - lj));
    }
    score[(long)in.b * ld_score + score_off + j] = sc;
}
void launch_score(const InstDesc* inst, int n_inst, const float* Ap, int d, const float* l, const float* u,
                  const int8_t* S, long ld_state, int state_off, float* score, long ld_score, int score_off,
                  hipStream_t st) {
    if (n_inst <= 0) return;
    hipLaunchKernelGGL(k_score, dim3(cdiv(d, 256), n_inst), dim3(256), 0, st, inst, Ap, d, l, u, S, ld_state,
                       state_off, score, ld_score, score_off);
    MNB_HIP(hipGetLastError());
}
// Active constraint score (Section 3.4, multi-neuron constraint guided branching): the
// sensitivity of the bound to the constraints that involve neuron j, through its output and
// its input, s_j = |(gamma^T P)_j| + |(gamma^T Phat)_j| for unstable, unsplit j (v = P^T gamma and
// vhat = Phat^T gamma come from k_gamma_proj), times the layer's weight (the inverse split cost
// of cost adjusted branching, else 1); -inf elsewhere.
// w: this layer's weight of instance 0, instance i's at w[i * ldw] (ldw 0: one weight for all; w null: 1)
__global__ void k_acs_score(const InstDesc* inst, const float* v, const float* vh, int d, const float* l,
                            const float* u, const int8_t* S, long ld_state, int state_off, const float* w, int ldw,
                            float* score, long ld_score, int score_off) {
    const InstDesc in = inst[blockIdx.y];
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= d) return;
    const long so = (long)in.slot * ld_state + state_off + j;
    const float lj = l[so], uj = u[so];
    const long vo = (long)blockIdx.y * d + j;
    float sc = -INFINITY;
    const float wt = w ? w[(long)blockIdx.y * ldw] : 1.f;
    if (S[so] == 0 && lj < 0.f && uj > 0.f) sc = (fabsf(v[vo]) + fabsf(vh[vo])) * wt;
    score[(long)in.b * ld_score + score_off + j] = sc;
}
void launch_acs_score(const InstDesc* inst, int n_inst, const float* v, const float* vh, int d, const float* l,
                      const float* u, const int8_t* S, long ld_state, int state_off, const float* w, int ldw,
                      float* score, long ld_score, int score_off, hipStream_t st) {
    if (n_inst <= 0 || d <= 0) return;
    hipLaunchKernelGGL(k_acs_score, dim3(cdiv(d, 256), n_inst), dim3(256), 0, st, inst, v, vh, d, l, u, S, ld_state,
                       state_off, w, ldw, score, ld_score, score_off);
    MNB_HIP(hipGetLastError());
}
// the score at each subproblem's argmax (-inf where there is none)
__global__ void k_pick(const float* score, long ld, const int32_t* arg, int n, float* out) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b < n) out[b] = arg[b] >= 0 ? score[(long)b * ld + arg[b]] : -INFINITY;
}
void launch_pick(const float* score, long ld, const int32_t* arg, int n, float* out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pick, dim3(cdiv(n, 256)), dim3(256), 0, st, score, ld, arg, n, out);
    MNB_HIP(hipGetLastError());
}
// argmax per subproblem, ties to the lowest index; -1 if nothing finite
__global__ void k_argmax(const float* score, long ld, int n, int32_t* out) {
    const int b = blockIdx.x;
    float best = -INFINITY;
    int arg = -1;
    for (int j = threadIdx.x; j < n; j += 256) {
        float v = score[(long)b * ld + j];
        if (v > best) {
            best = v;
            arg = j;
        }
    }
    __shared__ float sv[256];
    __shared__ int si[256];
    sv[threadIdx.x] = best;
    si[threadIdx.x] = arg;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            float v2 = sv[threadIdx.x + w];
            int i2 = si[threadIdx.x + w];
            float v1 = sv[threadIdx.x];
            int i1 = si[threadIdx.x];
            if (i2 >= 0 && (i1 < 0 || v2 > v1 || (v2 == v1 && i2 < i1))) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = si[0];
}
void launch_argmax(const float* score, long ld, int n, int nb, int32_t* out, hipStream_t st) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_argmax, dim3(nb), dim3(256), 0, st, score, ld, n, out);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ upper bound (forward pass at x*)
__global__ void k_bits_to_x(const uint8_t* bits, const int32_t* row_slot, const int32_t* qid, const float* lo,
                            const float* hi, int d0, int M, float* X) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)M * d0) return;
    int r = (int)(idx / d0), j = (int)(idx - (long)r * d0);
    int q = qid[row_slot[r]];
    X[idx] = bits[idx] ? hi[(long)q * d0 + j] : lo[(long)q * d0 + j];
}
void launch_bits_to_x(const uint8_t* bits, const int32_t* row_slot, const int32_t* qid, const float* lo,
                      const float* hi, int d0, int M, float* X, hipStream_t st) {
    if (M <= 0) return;
    long tot = (long)M * d0;
    hipLaunchKernelGGL(k_bits_to_x, dim3(cdiv(tot, 256)), dim3(256), 0, st, bits, row_slot, qid, lo, hi, d0, M,
                       X);
    MNB_HIP(hipGetLastError());
}
__global__ void k_relu_inplace(float* X, long n) {
    long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) X[j] = fmaxf(X[j], 0.f);
}
void launch_relu_inplace(float* X, long n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_relu_inplace, dim3(cdiv(n, 256)), dim3(256), 0, st, X, n);
    MNB_HIP(hipGetLastError());
}
// ub_r = C_q[s] . logits_r + c0_q[s]
__global__ void k_spec_dot(const float* logits, int n_out, const RowDesc* rows, const int32_t* slots,
                           const int32_t* qid, const float* C, const float* c0, int S, int M, float* ub) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    RowDesc rd = rows[r];
    int q = qid[slots[rd.b]];
    const float* Cr = C + ((long)q * S + rd.j) * n_out;
    float s = c0[(long)q * S + rd.j];
    for (int k = 0; k < n_out; ++k) s += Cr[k] * logits[(long)r * n_out + k];
    ub[r] = s;
}
void launch_spec_dot(const float* logits, int n_out, const RowDesc* rows, const int32_t* slots,
                     const int32_t* qid, const float* C, const float* c0, int S, int M, float* ub,
                     hipStream_t st) {
    if (M <= 0) return;
    hipLaunchKernelGGL(k_spec_dot, dim3(cdiv(M, 128)), dim3(128), 0, st, logits, n_out, rows, slots, qid, C, c0,
                       S, M, ub);
    MNB_HIP(hipGetLastError());
}

// Spec folded into the last affine layer: Chat = C W, chat = C b + c0.
__global__ void k_spec_fold(const float* C, const float* c0, const float* W, const float* b, int S, int n_out,
                            int din, float* Chat, float* chat) {
    int s = blockIdx.y;
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    const float* Cs = C + (long)s * n_out;
    if (j < din) {
        float acc = 0.f;
        for (int k = 0; k < n_out; ++k) acc += Cs[k] * W[(long)k * din + j];
        Chat[(long)s * din + j] = acc;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float acc = c0[s];
        for (int k = 0; k < n_out; ++k) acc += Cs[k] * b[k];
        chat[s] = acc;
    }
}
void launch_spec_fold(const float* C, const float* c0, const float* W, const float* b, int S, int n_out,
                      int din, float* Chat, float* chat, hipStream_t st) {
    hipLaunchKernelGGL(k_spec_fold, dim3(cdiv(din, 256), S), dim3(256), 0, st, C, c0, W, b, S, n_out, din, Chat,
                       chat);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ misc
__global__ void k_fill(float* p, long n, float v) {
    long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) p[j] = v;
}
void launch_fill(float* p, long n, float v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(cdiv(n, 256)), dim3(256), 0, st, p, n, v);
    MNB_HIP(hipGetLastError());
}

// heuristic alpha (1 if u > -l else 0) for every set of a slot over one layer
__global__ void k_heuristic_alpha(const float* l, const float* u, long ld_state, int off, int d, float* alpha,
                                  long ld_param, int n_sets, int slot) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    long so = (long)slot * ld_state + off + j;
    float a = (u[so] > -l[so]) ? 1.f : 0.f;
    for (int s = 0; s < n_sets; ++s) alpha[((long)slot * n_sets + s) * ld_param + off + j] = a;
}
void launch_heuristic_alpha(const float* l, const float* u, long ld_state, int off, int d, float* alpha,
                            long ld_param, int n_sets, int slot, hipStream_t st) {
    hipLaunchKernelGGL(k_heuristic_alpha, dim3(cdiv(d, 256)), dim3(256), 0, st, l, u, ld_state, off, d, alpha,
                       ld_param, n_sets, slot);
    MNB_HIP(hipGetLastError());
}

// unstable neurons per (local subproblem, layer): l < 0 < u
__global__ void k_count_unstable(const int32_t* slots, int nb, const float* l, const float* u, long ld_state,
                                 int off, int d, int32_t* count) {
    int b = blockIdx.x;
    int slot = slots[b];
    int c = 0;
    for (int j = threadIdx.x; j < d; j += 256) {
        long so = (long)slot * ld_state + off + j;
        c += (l[so] < 0.f && u[so] > 0.f) ? 1 : 0;
    }
    __shared__ int sc[256];
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sc[threadIdx.x] += sc[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) count[b] = sc[0];
}
void launch_count_unstable(const int32_t* slots, int nb, const float* l, const float* u, long ld_state, int off,
                           int d, int32_t* count, hipStream_t st) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_count_unstable, dim3(nb), dim3(256), 0, st, slots, nb, l, u, ld_state, off, d, count);
    MNB_HIP(hipGetLastError());
}

// Row descriptors of an intermediate-bound pass: for local subproblem b, its
// unstable neurons in index order, lower rows (+e_j, instance 2k) then upper
// rows (-e_j, instance 2k+1), starting at row offset row0[b].
__global__ void k_build_rows(const int32_t* bs, const int32_t* slots, const int32_t* row0, const int32_t* inst0,
                             const float* l, const float* u, long ld_state, int off, int d, RowDesc* rows) {
    const int k = blockIdx.x;
    const int b = bs[k];
    const int slot = slots[b];
    const int base = row0[k];
    __shared__ int scan[256];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    // count of this subproblem's unstable neurons (rows per direction)
    int total = 0;
    for (int j = threadIdx.x; j < d; j += 256) {
        long so = (long)slot * ld_state + off + j;
        total += (l[so] < 0.f && u[so] > 0.f) ? 1 : 0;
    }
    scan[threadIdx.x] = total;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) scan[threadIdx.x] += scan[threadIdx.x + w];
        __syncthreads();
    }
    const int nu = scan[0];
    __syncthreads();
    for (int j0 = 0; j0 < d; j0 += 256) {
        const int j = j0 + threadIdx.x;
        int flag = 0;
        if (j < d) {
            long so = (long)slot * ld_state + off + j;
            flag = (l[so] < 0.f && u[so] > 0.f) ? 1 : 0;
        }
        scan[threadIdx.x] = flag;
        __syncthreads();
        for (int w = 1; w < 256; w <<= 1) {
            int v = threadIdx.x >= w ? scan[threadIdx.x - w] : 0;
            __syncthreads();
            scan[threadIdx.x] += v;
            __syncthreads();
        }
        if (flag) {
            const int pos = carry + scan[threadIdx.x] - 1;
            rows[base + pos] = RowDesc{b, inst0[k], j, 1};
            rows[base + nu + pos] = RowDesc{b, inst0[k] + 1, j, -1};
        }
        __syncthreads();
        if (threadIdx.x == 255) carry += scan[255];
        __syncthreads();
    }
}
void launch_build_rows(const int32_t* bs, int nk, const int32_t* slots, const int32_t* row0, const int32_t* inst0,
                       const float* l, const float* u, long ld_state, int off, int d, RowDesc* rows,
                       hipStream_t st) {
    if (nk <= 0) return;
    hipLaunchKernelGGL(k_build_rows, dim3(nk), dim3(256), 0, st, bs, slots, row0, inst0, l, u, ld_state, off, d,
                       rows);
    MNB_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ branch_split
// Copy per-slot arrays of the parents into the children (vector width chosen by alignment).
template <class T>
__global__ void k_copy_slots(const int32_t* src, const int32_t* dst, T* base, long elems_per_slot) {
    const int c = blockIdx.y;
    const T* s = base + (long)src[c] * elems_per_slot;
    T* d = base + (long)dst[c] * elems_per_slot;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < elems_per_slot; i += (long)gridDim.x * blockDim.x)
        d[i] = s[i];
}
void launch_copy_slots(const int32_t* src, const int32_t* dst, int n, void* base, long bytes_per_slot,
                       hipStream_t st) {
    if (n <= 0 || bytes_per_slot <= 0) return;
    if (bytes_per_slot % 16 == 0 && ((uintptr_t)base % 16) == 0) {
        long e = bytes_per_slot / 16;
        int gx = std::min(64, cdiv(e, 256));
        hipLaunchKernelGGL(k_copy_slots<int4>, dim3(gx, n), dim3(256), 0, st, src, dst, (int4*)base, e);
    } else if (bytes_per_slot % 4 == 0 && ((uintptr_t)base % 4) == 0) {
        long e = bytes_per_slot / 4;
        int gx = std::min(64, cdiv(e, 256));
        hipLaunchKernelGGL(k_copy_slots<int>, dim3(gx, n), dim3(256), 0, st, src, dst, (int*)base, e);
    } else {
        long e = bytes_per_slot;
        int gx = std::min(64, cdiv(e, 256));
        hipLaunchKernelGGL(k_copy_slots<char>, dim3(gx, n), dim3(256), 0, st, src, dst, (char*)base, e);
    }
    MNB_HIP(hipGetLastError());
}

__global__ void k_apply_split(const int32_t* child, const int32_t* off_j, const int32_t* sign, int n, float* l,
                              float* u, int8_t* S, long ld_state, float* beta, long ld_param, int n_sets) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    long so = (long)child[c] * ld_state + off_j[c];
    if (sign[c] > 0) {
        S[so] = -1;
        l[so] = fmaxf(l[so], 0.f);
    } else {
        S[so] = 1;
        u[so] = fminf(u[so], 0.f);
    }
    for (int s = 0; s < n_sets; ++s) beta[((long)child[c] * n_sets + s) * ld_param + off_j[c]] = 0.f;
}
void launch_apply_split(const int32_t* child, const int32_t* off_j, const int32_t* sign, int n, float* l, float* u,
                        int8_t* S, long ld_state, float* beta, long ld_param, int n_sets, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_apply_split, dim3(cdiv(n, 128)), dim3(128), 0, st, child, off_j, sign, n, l, u, S,
                       ld_state, beta, ld_param, n_sets);
    MNB_HIP(hipGetLastError());
}

}  // namespace mnb
