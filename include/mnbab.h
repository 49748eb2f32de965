/*
 * mnbab.h -- C ABI of the MI355X batched back-substitution engine for
 * multi-neuron-constraint guided branch-and-bound (MN-BaB, Ferrari et al.,
 * ICLR 2022, arXiv 2205.00263).
 *
 * The library bounds  min_{x in box} C f(x) + c0  for a ReLU network f
 * (Section 2.1, Eq. 1; the linear property is folded into an extra affine
 * layer) over many branch-and-bound subproblems at once, by back-substitution
 * (Section 3.1: Eq. 2 for affine layers, Eq. 5 for ReLU layers, Eq. 6 for the
 * input box) with optimisable ReLU slopes alpha, split multipliers beta
 * (Eq. 4) and multi-neuron-constraint multipliers gamma (Eq. 3).
 *
 * Conventions
 *  - Every call returns an int status: MNB_OK (0), MNB_PENDING (1) or a
 *    negative error code.  mnb_last_error() gives a thread-local message.
 *    No C++ exception crosses this boundary.
 *  - Unless stated otherwise pointers are HOST pointers owned by the caller
 *    and only read during the call (the library copies what it keeps).
 *    Output arrays are caller-allocated with the documented sizes.
 *  - Floating point data is IEEE float32, row-major; conv tensors are
 *    (C, H, W) flattened, weights [Co][Ci][k][k].
 *  - Device memory is allocated through the installed allocator (default:
 *    hipMalloc) and work runs on the installed stream (default: a stream the
 *    library creates).  Calls are synchronous with respect to the host unless
 *    stated otherwise: they return once their results are in host memory.
 *  - A device error, or a NaN/Inf reaching a bound, never produces a positive
 *    (unsound) lower bound: the affected lb is reported as -INFINITY.
 */
#ifndef MNBAB_H
#define MNBAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define MNB_OK 0
#define MNB_PENDING 1
#define MNB_EINVAL (-1)   /* invalid argument or shape; nothing was written  */
#define MNB_ENOMEM (-2)   /* device allocation failed or capacity exhausted  */
#define MNB_EDEVICE (-3)  /* HIP runtime / kernel error                      */
#define MNB_ETIMEOUT (-4)
#define MNB_ESTATE (-5)   /* call not valid in the object's current state    */

const char* mnb_last_error(void);

/* ------------------------------------------------------------------ device plumbing */
/* Allocator hooks (e.g. a framework's caching allocator).  alloc(bytes, ctx)
 * returns a device pointer or NULL; free(ptr, ctx) releases it.  Passing NULL
 * functions restores hipMalloc/hipFree.  Install before creating objects. */
typedef void* (*mnb_alloc_fn)(size_t bytes, void* ctx);
typedef void (*mnb_free_fn)(void* ptr, void* ctx);
int mnb_set_allocator(mnb_alloc_fn alloc, mnb_free_fn free_fn, void* ctx);
/* Stream the library launches on (a hipStream_t cast to void*); NULL restores
 * the library's own stream.  Only default-priority streams are supported. */
int mnb_set_stream(void* hip_stream);

/* ------------------------------------------------------------------ network */
enum { MNB_INPUT = 0, MNB_FC = 1, MNB_CONV = 2, MNB_RELU = 3, MNB_ADD = 4, MNB_BN = 5, MNB_AVGPOOL = 6 };

/* One node of the network DAG (Section 2.1: affine layers zhat = W z + b,
 * ReLUs z = max(0, zhat); convolutional and residual layers as the paper's
 * networks use them, Tables 4-5).  Nodes are topologically ordered; node 0 is
 * MNB_INPUT with out_chw = input shape.  src (and src2 for MNB_ADD) index
 * earlier nodes.  MNB_FC: W [dout][din], b [dout], din = size of src.
 * MNB_CONV: W [Co][Ci][k][k], b [Co], stride, pad (zero padding), output
 * shape derived from the input shape.  MNB_RELU follows an MNB_FC, MNB_CONV
 * or MNB_ADD node; MNB_ADD joins two affine nodes of equal shape.  The last
 * node must be MNB_FC (the logits). in_chw/out_chw are checked when nonzero.
 * Batch normalisation and average pooling (Section 2.1 lists both among the
 * layers the method covers; both are affine): MNB_BN, y = gamma (x - mean) /
 * sqrt(var + eps) + beta per channel with W = [gamma | beta | mean | var]
 * (4 x C floats) and eps, must directly follow an MNB_FC or MNB_CONV node that
 * has no other consumer and is folded into that node's weights and bias;
 * MNB_AVGPOOL (k, stride, pad; the mean over each k x k window with the zero
 * padding counted, divisor k^2) becomes a convolution with 1/k^2 between equal
 * channels.  Node indices of the other entry points (kernel-level calls,
 * timer) count the nodes after this translation: MNB_BN nodes removed. */
typedef struct {
    int kind;
    int src;
    int src2;
    int in_chw[3];
    int out_chw[3];
    int k, stride, pad;
    const float* W;
    const float* b;
    float eps;
} mnb_layer;

typedef struct mnb_net mnb_net;
/* Copies the weights to the device.  Returns MNB_EINVAL for an unsupported
 * graph or inconsistent shapes. */
int mnb_net_create(const mnb_layer* layers, int n_layers, mnb_net** out);
void mnb_net_destroy(mnb_net* net);
/* Number of ReLU layers and their widths (caller array of n_relu ints). */
int mnb_net_info(const mnb_net* net, int* n_relu, int* relu_sizes, int* d_in, int* d_out);
/* Direct cost of a split in each ReLU layer (Appendix B, the cost model of cost
 * adjusted branching, Section 3.4): for a split in layer k, the sum over the
 * later layers i (the nodes after the input, in order) of 2 d_i C_i, where d_i
 * is layer i's output width and C_i the sum of the back-substitution costs c_j
 * of the layers before i: d_j + p_j for a ReLU layer with p_j multi-neuron
 * constraints, the weight count for a fully connected layer, d_j k_j^2 for a
 * convolution, and d_j for a residual addition (the appendix lists no cost for
 * it).  layers: the node list of mnb_net_create (only kinds, src and shapes
 * are read; no device work, so the call also works without a GPU);
 * mnc_counts [n_relu] (nullable: all 0, else each >= 0); costs [n_relu] out.
 * 1 / cost per layer is the layer_weight of mnb_branch_scores. */
int mnb_split_costs(const mnb_layer* layers, int n_layers, const int32_t* mnc_counts, double* costs);

/* ------------------------------------------------------------------ multi-neuron constraints */
/* Constraints  P z + Phat zhat <= p  over the output z and input zhat of ReLU
 * layer `layer` (Eq. 3), e rows in CSR form over that layer's neurons:
 * row_ptr [e+1], col [nnz], P [nnz], Phat [nnz], p [e]. */
typedef struct {
    int layer;
    int e;
    const int32_t* row_ptr;
    const int32_t* col;
    const float* P;
    const float* Phat;
    const float* p;
} mnb_mnc;

/* Constraint generator (host only, no device work).  The paper takes its
 * multi-neuron constraints from PRIMA (Section 3.1); this library generates
 * constraints of the same form from the exact convex hull of the graph of
 * three ReLUs over an input polytope Q = {v : s . v >= lb_s} given by
 * octahedral bounds on the 26 directions s in {-1,0,1}^3 \ {0}, listed in
 * lexicographic order of (s0, s1, s2) with -1 < 0 < 1: relu is linear on each
 * orthant, so the hull is that of the points (v, relu(v)) over the vertices v
 * of Q intersected with each orthant; facets come from the double description
 * method, each offset is reset to the maximum of its facet over those points
 * (valid whatever the rounding), and facets that involve one neuron only are
 * dropped.  lb [26]; out [max_out][7] = (Phat[3], P[3], p) per constraint
 * Phat . zhat + P . z <= p, normals scaled to max |coefficient| = 1, in the
 * lexicographic order of their normals; *n_out <= max_out written.  No
 * constraints (n_out 0) when the points do not span 6 dimensions. */
int mnb_relu_hull(const double* lb, int max_out, double* out, int* n_out);

/* ------------------------------------------------------------------ problems */
/* (mnb_octahedral_bounds / mnb_mnc_generate below generate constraints on the
 * device for a query's root.) */
/* A problem is a device-resident pool of `capacity` subproblem slots on one
 * network; every query added to it has n_spec spec rows.  max_mnc bounds the
 * number of MNC rows per ReLU layer of any query (0: no MNCs). */
typedef struct mnb_problem mnb_problem;
int mnb_problem_create(const mnb_net* net, int n_spec, int64_t capacity, int max_mnc,
                       mnb_problem** out);
void mnb_problem_destroy(mnb_problem* pb);

/* bound_init: add a query and bound its root with the DeepPoly pass that
 * precedes optimisation (Section 4 setup): heuristic alpha (1 if u > -l else
 * 0), beta = gamma = 0; ReLU layer 0 from the exact interval of the first
 * affine layer; later layers by back-substitution of the rows +-e_j of the
 * neurons an interval pass does not prove stable, intersected with that
 * interval.  x_lo/x_hi [d0]: the input box (the L-infinity ball of radius eps
 * around x0, clipped to the valid range).  C [n_spec][d_out], c0 [n_spec]:
 * spec rows, bounded as C f(x) + c0.  mnc: n_mnc constraint sets (may be
 * NULL), used by later bound_optimize calls through gamma.  Outputs: root
 * subproblem id, lb [n_spec], ub [n_spec] (ub = spec at the input minimising
 * each row's concretisation, Section 3.1 "Upper Bounding"). */
int bound_init(mnb_problem* pb, const float* x_lo, const float* x_hi, const float* C,
               const float* c0, const mnb_mnc* mnc, int n_mnc, int64_t* root_id, float* lb,
               float* ub);

/* branch_split: two children per (parent, ReLU layer, neuron) (Section 3.2,
 * "Enforcing Splits"): each copies its parent's state and parameters; the
 * split entry of S (Eq. 4) is -1 (positive phase, zhat >= 0) in the first
 * child and +1 (negative phase) in the second, the neuron's bound is
 * tightened to the phase, its beta is reset to 0, and ReLU layers after the
 * split layer are marked for recomputation at the next bound_optimize.
 * child [2n]: ids, positive child first.  Parents stay valid. */
int branch_split(mnb_problem* pb, const int64_t* parent, const int32_t* layer,
                 const int32_t* neuron, int n, int64_t* child);

typedef struct {
    int steps;             /* Adam updates (evaluations = steps + 1)                 */
    float lr, beta1, beta2, eps;
    int recompute_intermediate; /* 1: recompute layers after pending splits (Sec. 3.2) */
    int ckpt_stride;       /* adjoint checkpoint stride over ReLU layers (>=1); 0 = auto */
    size_t mem_budget;     /* bytes of device workspace per call; 0 = default        */
} mnb_opt_cfg;
void mnb_opt_cfg_default(mnb_opt_cfg* cfg);

/* bound_optimize: optimise (alpha, beta, gamma) of n subproblems by projected
 * Adam ascent (Section 3.1, last paragraphs) with the hand-written adjoint of
 * back-substitution; one parameter set per (subproblem, objective layer,
 * direction), shared by the rows of that objective.  Each evaluation first
 * recomputes, in ascending order, the intermediate bounds of the ReLU layers
 * after the subproblem's earliest pending split (rows: neurons unstable at
 * call start; new bounds are intersected with the old), then bounds the spec
 * rows.  lb/ub [n][n_spec]: best lb over the evaluations (and never below the
 * subproblem's previous lb) and the spec at that evaluation's minimiser.
 * branch_layer/branch_neuron [n] (nullable): the unstable, unsplit neuron
 * with the largest sum over spec rows of |a'_j| * (-u_j l_j / (u_j - l_j))
 * at the last evaluation (-1 if none). */
int bound_optimize(mnb_problem* pb, const int64_t* ids, int n, const mnb_opt_cfg* cfg, float* lb,
                   float* ub, int32_t* branch_layer, int32_t* branch_neuron);

/* bound_optimize in steps, for callers that interleave optimisation with other
 * work (a scheduler advancing batches one Adam step at a time) or time single
 * steps.  bound_optimize(cfg) is exactly begin(cfg), cfg->steps calls of step,
 * then end.  begin validates the ids, counts the neurons each subproblem
 * recomputes (unstable at this point), plans the passes and resets the Adam
 * moments; cfg->steps = 0 plans an evaluation only (step then returns
 * MNB_ESTATE).  step runs one evaluation (recomputed intermediate bounds, then
 * the spec rows; best lb per row kept), its adjoint and one projected Adam
 * update with bias correction for the session's own step count.  end runs the
 * last evaluation, the upper bound and the outputs of bound_optimize, updates
 * the subproblems' reported lb and frees the session; if end fails the session
 * stays valid for mnb_opt_session_destroy.  A session owns its workspace, so
 * other calls on the problem may run between steps, but the session's
 * subproblems must not be released, split or optimised elsewhere until end.
 * One session per thread at a time; sessions on one problem are serialised
 * by the problem's lock. */
typedef struct mnb_opt_session mnb_opt_session;
int bound_optimize_begin(mnb_problem* pb, const int64_t* ids, int n, const mnb_opt_cfg* cfg,
                         mnb_opt_session** out);
int bound_optimize_step(mnb_opt_session* s);
int bound_optimize_end(mnb_opt_session* s, float* lb, float* ub, int32_t* branch_layer,
                       int32_t* branch_neuron);
void mnb_opt_session_destroy(mnb_opt_session* s);

/* Read back a subproblem's intermediate bounds of ReLU layer `layer`
 * (l, u [d_layer]) and split diagonal S (int8 [d_layer], may be NULL). */
int mnb_get_bounds(mnb_problem* pb, int64_t id, int layer, float* l, float* u, int8_t* S);
/* Read / write a parameter set of a subproblem: set 0 = spec rows, set
 * 2m-1 / 2m = lower / upper bounds of ReLU layer m >= 1.  alpha, beta
 * [sum of ReLU widths] (layers below the set's objective are used), gamma
 * [n_relu * max_mnc].  Any pointer may be NULL. */
int mnb_get_params(mnb_problem* pb, int64_t id, int set, float* alpha, float* beta, float* gamma);
int mnb_set_params(mnb_problem* pb, int64_t id, int set, const float* alpha, const float* beta,
                   const float* gamma);
/* Gradient of a set's objective (sum of its rows' lower bounds) with respect
 * to the set's alpha, beta and gamma at the subproblem's current parameters
 * and bounds (the adjoint used by bound_optimize; l/u are not modified).
 * lb_rows [rows of the set] (nullable), g_alpha/g_beta [sum of ReLU widths],
 * g_gamma [n_relu * max_mnc]; each nullable.  Returns the row count in *rows. */
int mnb_bound_grad(mnb_problem* pb, int64_t id, int set, int* rows, float* lb_rows, float* g_alpha,
                   float* g_beta, float* g_gamma);
/* The same two calls on DEVICE pointers (for callers that keep the parameters
 * in device memory, e.g. behind torch.autograd.Function): mnb_set_params_device
 * copies alpha/beta/gamma device-to-device on the library stream;
 * mnb_bound_grad_device writes lb_rows (capacity: n_spec for set 0, else the
 * width of the set's ReLU layer), g_alpha, g_beta and g_gamma into device
 * arrays on the library stream.  Both return once the copies are done; the
 * caller orders its own stream's writes before the call (same stream via
 * mnb_set_stream, or a synchronisation). */
int mnb_set_params_device(mnb_problem* pb, int64_t id, int set, const float* alpha, const float* beta,
                          const float* gamma);
int mnb_bound_grad_device(mnb_problem* pb, int64_t id, int set, int* rows, float* lb_rows, float* g_alpha,
                          float* g_beta, float* g_gamma);
/* Branching scores of Section 3.4 from the multi-neuron constraints' Lagrange
 * parameters: the active constraint score of neuron j of ReLU layer i,
 * s_ij = |(gamma^T P)_j| + |(gamma^T Phat)_j| with gamma of set 0 (the spec
 * rows) as it stands, for every unstable (l < 0 < u), unsplit neuron; with
 * layer_weight [n_relu] (nullable: all 1; each finite and > 0) multiplied by
 * layer_weight[i], which with the inverse split costs of Appendix B is cost
 * adjusted branching (mnb_split_costs).  scores [n][sum of ReLU widths] (host, nullable; -inf
 * for non-candidates); branch_layer/branch_neuron [n] (nullable): the highest
 * score, ties to the lowest (layer, neuron), -1 if the subproblem has no
 * candidate.  MNB_EINVAL if the problem has no multi-neuron constraints or
 * n > 65535.  Parameters and bounds are not modified. */
int mnb_branch_scores(mnb_problem* pb, const int64_t* ids, int n, const float* layer_weight, float* scores,
                      int32_t* branch_layer, int32_t* branch_neuron);
/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): mnb_branch_scores
 * with every device buffer (ids, instance descriptors, layer weights, the
 * projections gamma^T P and gamma^T Phat, the scores and the argmax) carved
 * from a fixed device array of MNB_NOALLOC_SCRATCH_BYTES that the library
 * holds on each GPU it runs on until the process ends; no hipMalloc, hipFree
 * or allocating library routine is called.  Same arguments, results and
 * errors as mnb_branch_scores, bit for bit (the same kernels), except that
 * layer_weight is [n_relu] only, and MNB_EINVAL when the call needs more than
 * the array: 3 n (sum of ReLU widths) floats plus a few bytes per subproblem
 * (e.g. n <= 89 for the ConvBig shape).  Every scratch byte a call reads it
 * first writes.  Calls of one process are serialised on a host mutex and are
 * complete when they return; calls that overlapped on one GPU would race on
 * its array. */
#define MNB_NOALLOC_SCRATCH_BYTES (64u << 20)
int mnb_branch_scores_noalloc(mnb_problem* pb, const int64_t* ids, int n, const float* layer_weight,
                              float* scores, int32_t* branch_layer, int32_t* branch_neuron);
/* The alpha-contribution branching score that bound_optimize's branch_layer /
 * branch_neuron choose by (Section 3.2 splits an unstable ReLU; the score reads
 * the bound's sensitivity to each unstable, unsplit neuron times the height of
 * its triangle relaxation, Eq. 5): s_ij = sum over spec rows of |a'_j| *
 * (-u_j l_j / (u_j - l_j)), with a' the spec rows' coefficients on ReLU layer i
 * evaluated at the subproblems' current parameters (set 0) and bounds (no
 * recompute, nothing is written).  Right after bound_optimize these are the
 * parameters and bounds of its last evaluation, so the choice is the one it
 * returned.  scores [n][sum of ReLU widths] (host, nullable; -inf for
 * non-candidates); branch_layer/branch_neuron [n] (nullable): the highest score,
 * ties to the lowest (layer, neuron), -1 without a candidate.  MNB_EINVAL for
 * duplicate or invalid ids or n > 65535. */
int mnb_contribution_scores(mnb_problem* pb, const int64_t* ids, int n, float* scores,
                            int32_t* branch_layer, int32_t* branch_neuron);
/* Multi-neuron constraint generation on the device (the input of Eq. 3 that
 * the paper takes from PRIMA, Section 3.1).  mnb_octahedral_bounds: for the
 * groups [n][3] of neurons of ReLU layer `layer`, the lower bounds lb [n][26]
 * of s . zhat over the group for the 26 directions of mnb_relu_hull (same
 * order), by back-substitution of the rows sum_t s_t e_{g_t} on the layer's
 * input with the subproblem's parameters of the set bounding that layer from
 * below (heuristic alpha and beta = gamma = 0 right after bound_init), without
 * rounding margin.  mnb_mnc_generate: the constraints of every ReLU layer of
 * the subproblem's query from its current bounds: unstable neurons ordered by
 * the height -l u / (u - l) of their triangle (largest first, ties by index) in
 * consecutive disjoint triples; per group its octahedral bounds, then the
 * ReLU hull constraints of mnb_relu_hull on the host, group by group until cap
 * constraints per layer; coefficients are stored in float32 with each offset
 * recomputed for the rounded coefficients over the hull's vertices and
 * rounded up (the stored constraint stays valid).  The query's constraint sets
 * are replaced and gamma of the subproblem is reset to 0; e_out [n_relu]
 * (nullable) receives the counts.  Call it on a query's root before branching:
 * MNB_ESTATE if other subproblems of the query exist, MNB_EINVAL if the problem
 * has max_mnc = 0 or cap > max_mnc.  mnb_get_mnc reads a query's constraints of
 * one layer back (CSR as in mnb_mnc; arrays sized max_mnc + 1 / 4 max_mnc /
 * max_mnc, each nullable). */
int mnb_octahedral_bounds(mnb_problem* pb, int64_t id, int layer, const int32_t* groups, int n, float* lb);
int mnb_mnc_generate(mnb_problem* pb, int64_t id, int cap, int32_t* e_out);
int mnb_get_mnc(mnb_problem* pb, int64_t id, int layer, int* e, int32_t* row_ptr, int32_t* col, float* P,
                float* Phat, float* p);
/* Free subproblem slots. */
int mnb_release(mnb_problem* pb, const int64_t* ids, int n);
/* Slots in use / capacity. */
int mnb_problem_usage(const mnb_problem* pb, int64_t* used, int64_t* capacity);

/* ------------------------------------------------------------------ kernel-level entry points */
/* The back-substitution products on DEVICE pointers (row-major float32),
 * enqueued on the library stream; mnb_sync() waits for them.
 * fc_backsub:   C[M, din] (+)= A[M, dout] W[dout, din]      (Eq. 2, W of fc node `node`)
 * conv_backsub: C[M, Ci*Hi*Wi] (+)= transposed conv of A[M, Co*Ho*Wo] by conv node `node`
 * fc_forward / conv_forward: C = G W^T + b / conv(G) + b (the adjoint's forward products). */
int mnb_kernel_fc_backsub(const mnb_net* net, int node, const float* A, float* C, int M, int accumulate);
int mnb_kernel_conv_backsub(const mnb_net* net, int node, const float* A, float* C, int M, int accumulate);
int mnb_kernel_fc_forward(const mnb_net* net, int node, const float* G, float* C, int M);
int mnb_kernel_conv_forward(const mnb_net* net, int node, const float* G, float* C, int M);
int mnb_sync(void);

/* ------------------------------------------------------------------ kernel timer */
/* HIP events recorded on the library stream around every launch of one
 * kernel class while the timer runs.  node restricts timing to one network
 * node (-1: all nodes of that class).  Algorithmic work per launch: products
 * 2 * rows * (nonzero multiply-adds of the layer per row) flops; fold, relax
 * and concretise the bytes they must move (coefficient rows read/written);
 * MNB_T_BOTTOM (fused first-layer fold + transposed convolution +
 * concretisation + adjoint convolution) 4 * rows * (multiply-adds of the first
 * convolution) flops and, per row, 4 d1 bytes for each coefficient row read or
 * gradient / a' row written plus d0 x* bytes; MNB_T_BOTTOM_WIN (its
 * window-sparse form for rows whose objective is ReLU layer 1) 2 * rows *
 * (window positions x first-layer channels x taps) flops, doubled with the
 * adjoint.  Calls without rows (nothing launched) are not counted. */
enum { MNB_T_FC_BACKSUB = 1, MNB_T_CONV_BACKSUB = 2, MNB_T_FC_FORWARD = 3, MNB_T_CONV_FORWARD = 4,
       MNB_T_FOLD = 5, MNB_T_RELAX = 6, MNB_T_CONCRETIZE = 7, MNB_T_BOTTOM = 8,
       MNB_T_BOTTOM_WIN = 9 };
int mnb_timer_begin(int kind, int node);
/* Stop, wait for the stream and report launches, summed duration (ms), and
 * summed algorithmic flops and bytes of the timed launches. */
int mnb_timer_end(int64_t* launches, double* ms, double* flops, double* bytes);

/* ------------------------------------------------------------------ kernel variants */
/* Not an operation of the method: several kernels compute the same products
 * (Eq. 2, Eq. 5, Eq. 6 and their adjoints) to FP32 rounding, and the library
 * picks the fastest for each layer shape.  A set bit forces the more general
 * variant of one step for all later calls in this process (the mask is
 * process-wide; set it only between calls, not while another thread is in the
 * library):
 *   MNB_VAR_VALU_BOTTOM      fused first layer on the VALU kernel instead of MFMA
 *   MNB_VAR_NO_TAP_CONVT     transposed convolution of small grids by stride phases
 *   MNB_VAR_NO_PAIR_CONV     forward convolution with one wavefront per row
 *   MNB_VAR_NO_ROW_CONV      convolutions through the LDS-staged gather GEMMs
 *   MNB_VAR_NO_WINDOW        window rows of ReLU layer 1 through the fused kernel
 *   MNB_VAR_NO_FUSED_BOTTOM  first layer by the generic back-substitution and concretisation
 *   MNB_VAR_NO_PATCH         intermediate-bound rows of convolution outputs as whole
 *                            layers instead of receptive-field windows
 *   MNB_VAR_NO_CONE          the adjoint of receptive-field rows on whole rows instead
 *                            of forward cones
 *   MNB_VAR_NO_FIRST_CONV    first-layer convolutions (stride 1, at most 4 input
 *                            channels) through the general kernels
 *   MNB_VAR_NO_WIN_CONV      forward convolutions through the gather GEMM instead of
 *                            the input-window kernel
 * The initial mask comes from the environment variables MNB_BOTTOM_VALU,
 * MNB_NO_TAP_CONVT, MNB_NO_PAIR_CONV, MNB_NO_ROW_CONV, MNB_NO_WIN_BOTTOM,
 * MNB_NO_FUSED_BOTTOM, MNB_NO_PATCH, MNB_NO_CONE, MNB_NO_FIRST_CONV and
 * MNB_NO_WIN_CONV (set: bit on).  The
 * receptive-field bits are read when a pass is planned (bound_init,
 * bound_optimize, bound_optimize_begin).  mnb_set_kernel_variants returns the
 * previous mask; neither call fails. */
enum { MNB_VAR_VALU_BOTTOM = 1, MNB_VAR_NO_TAP_CONVT = 2, MNB_VAR_NO_PAIR_CONV = 4, MNB_VAR_NO_ROW_CONV = 8,
       MNB_VAR_NO_WINDOW = 16, MNB_VAR_NO_FUSED_BOTTOM = 32, MNB_VAR_NO_PATCH = 64, MNB_VAR_NO_CONE = 128,
       MNB_VAR_NO_FIRST_CONV = 256, MNB_VAR_NO_WIN_CONV = 512 };
int mnb_set_kernel_variants(int mask);
int mnb_get_kernel_variants(void);

/* ------------------------------------------------------------------ serving */
/* A verification query for the server: box, spec and MNC sets as in
 * bound_init, plus a per-query wall-clock budget.  With mnc_cap > 0 and no
 * MNC sets given, the server generates them for the query's root on the device
 * (mnb_mnc_generate, at most mnc_cap <= 500 per ReLU layer). */
typedef struct {
    int net_index;         /* index into the nets the server was created with */
    const float* x_lo;
    const float* x_hi;
    const float* C;
    const float* c0;
    int n_spec;
    const mnb_mnc* mnc;
    int n_mnc;
    double timeout_s;
    int mnc_cap;
} mnb_query;

enum { MNB_VERIFIED = 1, MNB_FALSIFIED = 2, MNB_UNKNOWN = 3, MNB_TIMEOUT = 4 };
/* Why a query ended UNKNOWN (or TIMEOUT). */
enum { MNB_R_NONE = 0, MNB_R_NO_SPLIT = 1 /* a leaf with no unstable, unsplit neuron left */,
       MNB_R_QUEUE_CAP = 2 /* its own queue_cap of live subproblems */,
       MNB_R_MEMORY = 3 /* alone on the server, its tree outgrew the memory budget */,
       MNB_R_ERROR = 4 /* a library error (see the server's error text) */, MNB_R_TIME = 5 };

typedef struct {
    int verdict;           /* MNB_VERIFIED / MNB_FALSIFIED / MNB_UNKNOWN / MNB_TIMEOUT */
    float lb;              /* min over spec rows of the root's optimised lb        */
    int64_t subproblems;   /* subproblems bounded for this query                   */
    double t_submit, t_admit, t_done;  /* seconds on the server's clock            */
    int reason;            /* MNB_R_*                                              */
    int restarts;          /* times the query was preempted and started again      */
} mnb_result;

typedef struct {
    mnb_opt_cfg opt;       /* per-batch optimisation settings (opt.mem_budget 0:   */
                           /* a quarter of mem_budget per call)                    */
    int max_batch;         /* subproblems per engine step                          */
    int64_t queue_cap;     /* live subproblems per query before UNKNOWN            */
    size_t mem_budget;     /* device bytes of all slot pools and workspaces        */
    int64_t max_slots;     /* slots per pool at most (0: as many as mem_budget allows) */
} mnb_server_cfg;
void mnb_server_cfg_default(mnb_server_cfg* cfg);

typedef struct mnb_server mnb_server;
/* Continuous-batching server: a host thread admits queries as slots and the
 * memory budget allow, advances every live subproblem batch by one
 * bound_optimize call per iteration, and branches or retires subproblems
 * (lb > 0 on every spec row: verified; ub < 0: counterexample).
 * Memory: each (net, spec count, constraint use) has a slot pool that starts
 * small and doubles while the pools and the problems' workspaces stay within
 * mem_budget.  When a split finds no room its parent waits (parked, not
 * bounded again) and is split as soon as slots free up; parked splits take
 * precedence over admitting new queries.  If an iteration can neither bound
 * nor split anything, the most recently admitted query holding slots is
 * preempted (its subproblems released, the query queued again at the front
 * to start over, result.restarts counted); a query alone on the server whose
 * tree no longer fits ends UNKNOWN with reason MNB_R_MEMORY.  A query's own
 * queue_cap still ends it UNKNOWN (MNB_R_QUEUE_CAP).  Waiting queries time
 * out like live ones. */
int mnb_server_create(mnb_net* const* nets, int n_nets, const mnb_server_cfg* cfg,
                      mnb_server** out);
void mnb_server_destroy(mnb_server* srv);
/* Non-blocking, thread-safe.  MNB_EINVAL (nothing queued) for bad arrays, a bad
 * net index, more than 500 constraints per layer, or a query whose root and
 * first two children alone exceed mem_budget. */
int query_submit(mnb_server* srv, const mnb_query* q, uint64_t* ticket);
/* MNB_PENDING until the query is done; then MNB_OK and *out filled. */
int query_poll(mnb_server* srv, uint64_t ticket, mnb_result* out);

#ifdef __cplusplus
}
#endif
#endif /* MNBAB_H */
