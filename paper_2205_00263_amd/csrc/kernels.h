// Launchers of the HIP kernels (internal interface between the engine and the kernels).
#pragma once

#include "common.h"

namespace mnb {

// Geometry of one convolution node plus the device tables its kernels use.
struct ConvPhase {
    int rho_y, rho_x;   // residues (Y + pad) mod stride of this phase
    int Y0, X0;         // first output position of the phase
    int nY, nX;         // positions of the phase
    int Ty, Tx;         // taps of the phase
    int q0y, q0x;       // (Y0 + pad - rho)/stride
    const float* Wp;    // [Ty][Tx][Co][Ci] weights of the phase
    const float* Wpg;   // the same with K ordered (co / 16, ty, tx, co % 16) (Co % 16 == 0)
    const int2* ktab;   // [Ty*Tx*Co] {co*Ho*Wo - ty*Wo - tx, (ty<<16)|tx}
    const float* Wt;    // [Co/8][Ty*Tx][8][Ci] flipped taps for the input-window kernel (Co % 8 == 0)
};

struct ConvGeom {
    int Ci, Hi, Wi, Co, Ho, Wo, k, s, p;
    const float* W;     // [Co][Ci][k][k]
    const float* b;     // [Co]
    const int2* fwd_ktab;  // [k*k*Ci] {ci*Hi*Wi + ky*Wi + kx, (ky<<16)|kx}, K ordered (ky, kx, ci)
    const float* Wf;       // [Co][k*k*Ci] weights in that K order
    const float* Wg;       // [Co][k*k*Ci] weights with K ordered (ci / 16, ky, kx, ci % 16) (Ci % 16 == 0)
    const float* Wt;       // [Ci/8][k*k][8][Co] weights of the input-window kernel (Ci % 8 == 0)
    // stride 2 with four phases of equal grid and square taps T x T: their flipped taps side by
    // side, [Co/8][4][T*T][8][Ci] (Co % 8 == 0), for the transposed window kernel; else null
    const float* Wt4;
    int n_phase;
    ConvPhase ph[16];   // stride <= 4
};

// Rows held on forward cones (receptive-field rows): a forward convolution given a clip writes 0
// at every position of row r's output cone that lies outside the node, so that the next
// convolution reads those entries as padding.  Row r's cone origin on the node is
// (yo S - Q, xo S - Q) for its objective position (yo, xo) = (j mod HWobj) / Wobj, % Wobj.
struct ConeClip {
    const RowDesc* rows;       // null: no clip
    int H, W;                  // node
    int S, Q, HWobj, Wobj;
};
__device__ __forceinline__ void cone_origin(const ConeClip& k, long r, int& oy, int& ox) {
    const int pos = k.rows[r].j % k.HWobj;
    const int yo = pos / k.Wobj, xo = pos - yo * k.Wobj;
    oy = yo * k.S - k.Q;
    ox = xo * k.S - k.Q;
}

// ---- back-substitution products (Eq. 2) ----
// C[M, din] (+)= A[M, dout] * W[dout, din]
void launch_fc_backsub(const float* A, const float* W, float* C, int M, int dout, int din,
                       bool accumulate, hipStream_t st);
// C[M, Ci*Hi*Wi] (+)= conv-transpose of A[M, Co*Ho*Wo]
void launch_conv_backsub(const ConvGeom& g, const float* A, float* C, int M, bool accumulate,
                         hipStream_t st);
// Row-resident MFMA forms of the two convolution products, used by launch_conv_backsub /
// launch_conv_forward when a row fits in LDS; false (nothing launched) otherwise.
bool launch_conv_backsub_rows(const ConvGeom& g, const float* A, float* C, int M, bool accumulate,
                              hipStream_t st);
bool launch_conv_forward_rows(const ConvGeom& g, const float* G, float* C, int M, bool accumulate,
                              hipStream_t st);
// VALU forms for convolutions of stride 1 out of (forward) or into (transposed) at most 4
// channels with 3x3 filters; false (nothing launched) for other shapes.
bool launch_convT_first(const ConvGeom& g, const float* A, float* C, int M, bool accumulate, hipStream_t st);
bool launch_conv_first(const ConvGeom& g, const float* G, float* C, int M, bool accumulate, hipStream_t st,
                       const ConeClip* clip = nullptr);
// Forward convolution from input windows staged in LDS (8 input channels at a time, Co % 32 == 0,
// 3x3 / 1, 3x3 / 2 or 4x4 / 2 filters); false (nothing launched) for other shapes.
bool launch_conv_forward_win(const ConvGeom& g, const float* G, float* C, int M, bool accumulate, hipStream_t st,
                             const ConeClip* clip = nullptr);
// Transposed convolution by the same kernel, one stride phase at a time (each phase is a stride-1
// correlation of the coefficient grid with the phase's flipped taps; square phases of 2x2 or 3x3
// taps, Co % 8 == 0, Ci % 32 == 0); false (nothing launched) for other shapes.
bool launch_conv_backsub_win(const ConvGeom& g, const float* A, float* C, int M, bool accumulate, hipStream_t st);

// ---- forward products (adjoint and upper-bound evaluation) ----
// C[M, dout] = G[M, din] * W^T + b  (accumulate: C += ..., bias added either way)
void launch_fc_forward(const float* G, const float* W, const float* b, float* C, int M, int din,
                       int dout, bool accumulate, hipStream_t st);
void launch_conv_forward(const ConvGeom& g, const float* G, float* C, int M, bool accumulate,
                         hipStream_t st, const ConeClip* clip = nullptr);

// Relaxation of one neuron (the D / b-underline case table of Section 3.1 with
// the split matrix of Eq. 4): split first, then stable, then unstable.
struct NeuronRelax {
    float dpos, dneg, bneg;
    bool unstable;
};

__device__ __forceinline__ NeuronRelax neuron_relax(float l, float u, int s, float alpha) {
    NeuronRelax r;
    r.unstable = false;
    r.bneg = 0.f;
    if (s == -1) {
        r.dpos = r.dneg = 1.f;
    } else if (s == 1) {
        r.dpos = r.dneg = 0.f;
    } else if (l >= 0.f) {
        r.dpos = r.dneg = 1.f;
    } else if (u <= 0.f) {
        r.dpos = r.dneg = 0.f;
    } else {
        r.unstable = true;
        r.dpos = alpha;
        float w = u - l;
        r.dneg = u / w;
        r.bneg = -(u * l) / w;
    }
    return r;
}

// ---- elementwise / reduction kernels (relu.hip) ----
// Receptive-field ("patch") rows: on one node of a pass, every row is the window [C][P][P] of
// the node that its objective neuron j sees, with origin (y_j S - Q, x_j S - Q), where (y_j, x_j)
// is j's position (j mod HWobj) on the objective layer.  Entries outside the node are padding.
struct PatchGeom {
    int C, H, W;          // node shape
    int P, S, Q;          // window side, origin stride and offset
    int HWobj, Wobj;      // positions of the objective layer and its width
};

struct FoldArgs {
    float* A;             // [M, d] in: a (coef on z), out: ahat (coef on zhat)
    float* Ap;            // [M, d] out: a' (nullable)
    float* cpart;         // [M, ldcp] per-wave partial constants (written at col_off + j/64)
    int ldcp, col_off;
    const InstDesc* inst; int n_inst;
    const int32_t* slots; // local b -> global slot
    int M, d;
    // per-slot state (global slot index), layer offset already applied
    const float* l; const float* u; const int8_t* S; long ld_state;
    // parameters: base + (slot*n_sets + set)*ld_param + layer offset
    const float* alpha; const float* beta; long ld_param; int n_sets;
    // gamma projections (nullable): per instance [n_inst, d]
    const float* v; const float* vhat;
    const float* bias;    // [d] effective bias of the affine output feeding this ReLU
    // rows +-e_j on the output of a fully connected layer (Wsrc [dout, d]) folded directly:
    // a = sign W[j] is read from Wsrc instead of A, and c[r] = sign bias_obj[j] is written
    // (nullable: a is read from A)
    const float* Wsrc; const RowDesc* rows; float* c; const float* bias_obj;
    // receptive-field rows: per instance and neuron {D(a' >= 0), D(a' < 0), b-underline, a'} of the
    // instance's shared row [n_inst, d] (A holds windows of the deviation from it); rt_out
    // (nullable) receives that table from a fold of the shared rows (one row per instance)
    const float4* rt_in;
    float4* rt_out;
};
void launch_relu_fold(const FoldArgs& a, hipStream_t st);

struct RelaxArgs {
    float* G;             // [M, d] in: ghat (forward value at the ReLU input), out: g (at its output)
    const float* Ap;      // [M, d] a' of the same rows
    const InstDesc* inst; int n_inst;
    const int32_t* slots;
    int M, d;
    const float* l; const float* u; const int8_t* S; long ld_state;
    const float* alpha; long ld_param; int n_sets;
    // gradient outputs per instance [n_inst, ldg] at column offset goff
    float* d_alpha; float* d_beta; long ldg; long goff;
    float* gsum_hat; float* gsum_out;  // nullable, [n_inst, d] (for gamma)
    // row slices of the cone relaxation (kRowSlice rows each on the third grid dimension, so that
    // an instance's rows are spread over many wavefronts): slice z of instance i writes partial sums
    // at slot zoff[i] + z of part [zoff[n_inst]][3][d], which launch_relax_sum adds in slice order,
    // so every sum has an order fixed by the instance alone; n_slices: most slices of an instance
    const int* zoff; int n_slices; float* part;
};
constexpr int kRowSlice = 64;
void launch_relu_relax(const RelaxArgs& a, hipStream_t st);
// d_alpha, d_beta and the gamma sums from the slices' partial sums in a.part
void launch_relax_sum(const RelaxArgs& a, hipStream_t st);
void launch_relu_fold(const FoldArgs& a, hipStream_t st, const float* gp);

struct ConcArgs {
    int mode;              // 0: intermediate-bound rows (update l/u), 1: spec rows, 2: lb only
    float margin;          // rounding margin factor: 2^-20 for spec rows, 0 for intermediate rows
    const float* A;        // [M, d0] coefficients on the input
    const float* c;        // [M]
    const float* cpart; int ldcp, ncp;  // partial constants of the folds
    const RowDesc* rows; const int32_t* slots; const int32_t* qid;
    const float* lo; const float* hi;   // [n_query, d0]
    int M, d0;
    float* G0;             // [M, d0] x* (nullable)
    uint8_t* xbits;        // [M, d0] 1 where x* = hi (nullable)
    // mode 0
    float* l; float* u; long ld_state; int state_off;
    // mode 1
    float* lb_out; float* best; uint8_t* improved;
    // receptive-field rows (pg.P > 0): A holds windows [M, C0 P P] of each row's deviation from its
    // instance's shared row, whose input coefficients ush0 [n_inst, d0] and bound lbs [n_inst] are
    // added; G0 (dense [M, d0], already holding the shared row's x*) gets the window entries
    PatchGeom pg;
    const float* ush0; const float* lbs; int inst_base;
    int g0_dev;            // G0 holds the windows of x* - x*(shared row) [M, C0 P P] instead
};
void launch_concretize(const ConcArgs& a, hipStream_t st);
void launch_keep_best_x(const uint8_t* xbits, uint8_t* best_bits, const uint8_t* improved, int M, int d0,
                        hipStream_t st);

void launch_init_spec(const RowDesc* rows, int M, const int32_t* slots, const int32_t* qid, const float* Chat,
                      const float* chat, int S, int d, float* A, float* c, hipStream_t st);
void launch_init_fc(const RowDesc* rows, int M, const float* W, const float* bias_eff, int din, float* A,
                    float* c, bool write_c, hipStream_t st);
void launch_init_conv(const RowDesc* rows, int M, const ConvGeom& g, const float* bias_eff, float* A, float* c,
                      bool write_c, hipStream_t st);
void launch_init_oct(const int32_t* grp, int n_groups, int d, const float* bias, float* A, float* c,
                     hipStream_t st);

void launch_ibp_fc(const float* W, const float* b, const float* L, const float* U, float* Lo, float* Uo, int din,
                   int dout, hipStream_t st);
void launch_ibp_conv(const ConvGeom& g, const float* L, const float* U, float* Lo, float* Uo, hipStream_t st);
void launch_ibp_relu(const float* L, const float* U, const float* lk, const float* uk, float* Lo, float* Uo, int d,
                     hipStream_t st);
void launch_add2(const float* a, const float* b, float* o, long n, hipStream_t st);

struct AdamArgs {
    const InstDesc* inst; int n_inst;
    float* alpha; float* beta; long ld_param; int n_sets;
    float* m_alpha; float* v_alpha; float* m_beta; float* v_beta;   // [nb, n_sets, ld_param]
    const float* g_alpha; const float* g_beta; long ldg;            // [n_inst, ldg]
    int n_ab;              // alpha/beta entries of the set (prefix of the layer space)
    // current bounds and splits: alpha moves only on unstable neurons, beta only on split ones
    const float* l; const float* u; const int8_t* S; long ld_state;
    float* gamma; float* m_gamma; float* v_gamma; const float* g_gamma; long ld_gamma; int n_gamma;
    float lr, b1, b2, eps, bc1, bc2;
};
void launch_adam(const AdamArgs& a, hipStream_t st);

struct GammaArgs {
    const InstDesc* inst; int n_inst;
    const int32_t* qid;
    const float* gamma; long ld_gamma; int n_sets; int goff;   // this layer's gamma offset
    int d, e_cap, nnz_cap;
    const int* e_of;                                      // [n_query] constraints of this layer
    const int* colptr; const int* col_e; const float* col_P; const float* col_Ph;   // CSC per query
    const int* rowptr; const int* row_j; const float* row_P; const float* row_Ph;   // CSR per query
    const float* p;                                       // [n_query, e_cap]
    float* v; float* vhat; float* gp;                     // [n_inst, d], [n_inst, d], [n_inst]
};
void launch_gamma_proj(const GammaArgs& a, hipStream_t st);
void launch_gamma_grad(const GammaArgs& a, const float* gsum_hat, const float* gsum_out, float* g_gamma, long ldgg,
                       hipStream_t st);

void launch_score(const InstDesc* inst, int n_inst, const float* Ap, int d, const float* l, const float* u,
                  const int8_t* S, long ld_state, int state_off, float* score, long ld_score, int score_off,
                  hipStream_t st);
void launch_argmax(const float* score, long ld, int n, int nb, int32_t* out, hipStream_t st);
void launch_pick(const float* score, long ld, const int32_t* arg, int n, float* out, hipStream_t st);
void launch_acs_score(const InstDesc* inst, int n_inst, const float* v, const float* vh, int d, const float* l,
                      const float* u, const int8_t* S, long ld_state, int state_off, const float* w, int ldw,
                      float* score, long ld_score, int score_off, hipStream_t st);

void launch_bits_to_x(const uint8_t* bits, const int32_t* row_slot, const int32_t* qid, const float* lo,
                      const float* hi, int d0, int M, float* X, hipStream_t st);
void launch_relu_inplace(float* X, long n, hipStream_t st);
void launch_spec_dot(const float* logits, int n_out, const RowDesc* rows, const int32_t* slots, const int32_t* qid,
                     const float* C, const float* c0, int S, int M, float* ub, hipStream_t st);
void launch_spec_fold(const float* C, const float* c0, const float* W, const float* b, int S, int n_out, int din,
                      float* Chat, float* chat, hipStream_t st);
void launch_fill(float* p, long n, float v, hipStream_t st);
void launch_heuristic_alpha(const float* l, const float* u, long ld_state, int off, int d, float* alpha,
                            long ld_param, int n_sets, int slot, hipStream_t st);
void launch_count_unstable(const int32_t* slots, int nb, const float* l, const float* u, long ld_state, int off,
                           int d, int32_t* count, hipStream_t st);
void launch_build_rows(const int32_t* bs, int nk, const int32_t* slots, const int32_t* row0, const int32_t* inst0,
                       const float* l, const float* u, long ld_state, int off, int d, RowDesc* rows,
                       hipStream_t st);

// ---- patch rows (patch.hip) ----
void launch_init_conv_patch(const RowDesc* rows, int M, const float* W, const float* bias_eff, int per_co,
                            int HWobj, float* A, float* c, hipStream_t st);
void launch_relu_fold_patch(const FoldArgs& a, const PatchGeom& g, const RowDesc* rows, int inst_base,
                            hipStream_t st);
// shared rows' forward relaxation gs = D(U') ghs + b(U') per (instance, neuron)
void launch_relax_shared(const RelaxArgs& a, const float* ush, const float* ghs, float* gs, hipStream_t st);
// adjoint relaxation of rows held as cone deviations Gd (in place) with their a' deviation windows,
// in row slices (RelaxArgs)
void launch_relax_cone(const RelaxArgs& a, const PatchGeom& gw, const PatchGeom& gc, const RowDesc* rows,
                       const float* ush, const float* ghs, const float* apw, float* Gd, hipStream_t st);
// zero the cone entries of rows [0, M) outside the node (for cones not written by a clipped
// convolution)
void launch_cone_zero(const PatchGeom& gc, const RowDesc* rows, int M, float* Gd, hipStream_t st);
// dense rows out[r] = shared[instance of r] + (window entries of win[r], nullable)
void launch_patch_expand(const float* shared, const float* win, const RowDesc* rows, int M, int inst_base,
                         const PatchGeom& g, float* out, hipStream_t st);
void launch_copy_slots(const int32_t* src, const int32_t* dst, int n, void* base, long bytes_per_slot,
                       hipStream_t st);
void launch_apply_split(const int32_t* child, const int32_t* off_j, const int32_t* sign, int n, float* l, float* u,
                        int8_t* S, long ld_state, float* beta, long ld_param, int n_sets, hipStream_t st);

}  // namespace mnb
