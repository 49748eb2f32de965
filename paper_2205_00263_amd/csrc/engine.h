// Host-side engine objects behind the C ABI.
#pragma once

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mnbab.h"
#include "kernels.h"

namespace mnb {

// ---------------------------------------------------------------- device memory / stream
void* dalloc(size_t bytes);
void dfree(void* p);
hipStream_t stream();

// Grow-only named device buffers; growing synchronises the stream first.
struct Workspace {
    struct Buf {
        void* p = nullptr;
        size_t bytes = 0;
    };
    std::map<std::string, Buf> bufs;
    template <class T>
    T* get(const std::string& name, size_t count) {
        size_t bytes = count * sizeof(T);
        if (bytes == 0) bytes = 16;
        Buf& b = bufs[name];
        if (b.bytes < bytes) {
            if (b.p) {
                MNB_HIP(hipStreamSynchronize(stream()));
                dfree(b.p);
            }
            size_t nb = bytes + bytes / 8 + 256;
            b.p = dalloc(nb);
            b.bytes = nb;
        }
        return (T*)b.p;
    }
    size_t total() const {
        size_t t = 0;
        for (auto& kv : bufs) t += kv.second.bytes;
        return t;
    }
    ~Workspace() {
        for (auto& kv : bufs)
            if (kv.second.p) dfree(kv.second.p);
    }
};

// Kernel timer: events around launches of one kernel class (see mnb_timer_begin).
struct TimerScope {
    bool on = false;
    hipEvent_t e0{}, e1{};
    TimerScope(int kind, int node, double flops, double bytes);
    ~TimerScope();
};

struct NetNode {
    int kind = 0, src = -1, src2 = -1;
    int C = 0, H = 0, W = 0, size = 0;
    int k = 0, stride = 1, pad = 0;
    float* Wd = nullptr;
    float* bd = nullptr;
    ConvGeom geom{};
    int relu_m = -1;
    double macs_per_row = 0;   // nonzero multiply-adds of the layer for one row
};

// Receptive-field rows of the intermediate bounds of one ReLU layer that a convolution feeds,
// when every node below that convolution is a convolution or a ReLU: for each node of the pass
// the window geometry of its rows, for each convolution the convolution between windows
// (padding 0: a window holds every tap its outputs read) and its multiply-adds per row.
//
// The adjoint of such rows runs on forward cones: a row's forward values (Appendix of the
// adjoint: x* pushed through the row's linearisation) differ from its set's shared row only on
// the positions its input window reaches going up, the cone; per node its geometry fc (origin
// y_j S - Q, side P) and per convolution the convolution between cones (no bias: deviations).
struct PatchPlan {
    bool ok = false;
    int top = -1;                  // the objective convolution's input node
    std::vector<PatchGeom> g;      // per node index
    std::vector<ConvGeom> conv;    // per node index (convolution nodes of the pass)
    std::vector<double> macs;      // per node index
    int max_width = 0;
    int width(int n) const { return g[n].C * g[n].P * g[n].P; }
    bool cone_ok = false;          // adjoint on cones (else on whole rows)
    std::vector<PatchGeom> fc;     // per node index
    std::vector<ConvGeom> fconv;   // per node index (convolution nodes)
    std::vector<double> fmacs;     // per node index
    int cone_width(int n) const { return fc[n].C * fc[n].P * fc[n].P; }
};

}  // namespace mnb

struct mnb_net {
    std::vector<mnb::NetNode> nodes;
    std::vector<int> relus, relu_d, relu_off;
    std::vector<float*> relu_bias;   // effective bias of each ReLU's input node, expanded [d]
    std::vector<void*> owned;
    int total_d = 0, d0 = 0, n_out = 0, last = 0, max_width = 0;
    bool bottom_ok = false;   // first layer is a small conv of the input feeding ReLU layer 0
    bool win_ok = false;      // ReLU layer 1 is fed by a conv of ReLU layer 0 the window kernel takes
    std::vector<mnb::PatchPlan> patch;   // per ReLU layer
    ~mnb_net();
};

namespace mnb {
size_t problem_slot_bytes(const mnb_problem* pb);
void problem_grow(mnb_problem* pb, int64_t capacity);
// Active constraint branching adjusted by the split costs of Appendix B (Section 3.4) for the
// subproblems ids: chosen layer / neuron (-1 without a candidate) and its score per subproblem.
// Returns an MNB status code (MNB_EINVAL without multi-neuron constraints).
int branch_acs_cab(mnb_problem* pb, const int64_t* ids, int n, int32_t* layer, int32_t* neuron, float* best);
}  // namespace mnb

struct mnb_problem {
    mnb_net* net = nullptr;
    int S = 0, R = 0, n_sets = 0, e_cap = 0;
    int64_t cap = 0;
    long ld_state = 0, ld_param = 0, ld_gamma = 0;
    // per-slot device arrays
    float *l = nullptr, *u = nullptr, *alpha = nullptr, *beta = nullptr, *gamma = nullptr;
    int8_t* S_ = nullptr;
    int32_t* qid = nullptr;
    float* lb = nullptr;   // [cap, S] reported lb
    // host mirrors
    std::vector<int> recompute_from, slot_query;
    std::vector<char> used;
    std::vector<int64_t> free_list;
    int64_t n_used = 0;
    // queries (device, growable)
    int n_query = 0, q_cap = 0;
    float *lo = nullptr, *hi = nullptr, *Chat = nullptr, *chat = nullptr, *C = nullptr, *c0 = nullptr;
    // MNC per layer: arrays [q_cap][...] per layer
    struct MncLayer {
        int* e_of = nullptr;
        int *colptr = nullptr, *col_e = nullptr, *rowptr = nullptr, *row_j = nullptr;
        float *col_P = nullptr, *col_Ph = nullptr, *row_P = nullptr, *row_Ph = nullptr, *p = nullptr;
    };
    std::vector<MncLayer> mnc;
    std::vector<std::vector<int32_t>> q_mnc_e;   // host: constraints per ReLU layer of each query
    int nnz_cap = 0;
    bool has_mnc = false;
    std::vector<void*> owned;
    mnb::Workspace ws;
    std::mutex mu;
    ~mnb_problem();
};
