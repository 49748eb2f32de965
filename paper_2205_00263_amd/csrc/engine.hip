// Host engine: network and problem state on the device, the back-substitution
// passes, their adjoint, and the C ABI of include/mnbab.h.
#include "engine.h"
#include "bottom.h"
#include "hull.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <numeric>
#include <set>

using namespace mnb;

// =====================================================================================
// errors, allocator, stream
// =====================================================================================
namespace mnb {
static thread_local std::string t_err;
void set_error(int code, const std::string& msg) {
    (void)code;
    t_err = msg;
}

static mnb_alloc_fn g_alloc = nullptr;
static mnb_free_fn g_free = nullptr;
static void* g_ctx = nullptr;
static hipStream_t g_user_stream = nullptr;
static hipStream_t g_own_stream = nullptr;
static std::mutex g_mu;

void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (g_alloc) {
        p = g_alloc(bytes, g_ctx);
        if (!p) throw Error{MNB_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes"};
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess)
            throw Error{MNB_ENOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e)};
    }
    return p;
}
void dfree(void* p) {
    if (!p) return;
    if (g_free)
        g_free(p, g_ctx);
    else
        (void)hipFree(p);
}
hipStream_t stream() {
    if (g_user_stream) return g_user_stream;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_own_stream) MNB_HIP(hipStreamCreateWithFlags(&g_own_stream, hipStreamNonBlocking));
    return g_own_stream;
}

// Host-to-device copy that has completed when it returns (sources are often temporaries).
static void h2d(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    MNB_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream()));
    MNB_HIP(hipStreamSynchronize(stream()));
}

template <class T>
static T* upload(const T* h, size_t n, std::vector<void*>* owned) {
    T* d = (T*)dalloc(std::max<size_t>(n * sizeof(T), 16));
    if (n) h2d(d, h, n * sizeof(T));
    if (owned) owned->push_back(d);
    return d;
}
static void sync() { MNB_HIP(hipStreamSynchronize(stream())); }
}  // namespace mnb

// ---------------------------------------------------------------- kernel timer
namespace mnb {
struct TimerState {
    int kind = 0, node = -1;
    bool running = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    double flops = 0, bytes = 0;
};
static TimerState g_timer;
static thread_local int t_timer_node = -1;

TimerScope::TimerScope(int kind, int node, double flops, double bytes) {
    if (!g_timer.running || g_timer.kind != kind || (g_timer.node >= 0 && g_timer.node != node)) return;
    if (flops <= 0.0 && bytes <= 0.0) return;   // no rows: nothing is launched
    if (g_timer.used == g_timer.ev.size()) {
        hipEvent_t a, b;
        MNB_HIP(hipEventCreate(&a));
        MNB_HIP(hipEventCreate(&b));
        g_timer.ev.push_back({a, b});
    }
    e0 = g_timer.ev[g_timer.used].first;
    e1 = g_timer.ev[g_timer.used].second;
    g_timer.used++;
    g_timer.flops += flops;
    g_timer.bytes += bytes;
    on = true;
    MNB_HIP(hipEventRecord(e0, stream()));
}
TimerScope::~TimerScope() {
    if (on) (void)hipEventRecord(e1, stream());
}
}  // namespace mnb

#define API_BEGIN try {
#define API_END                                  \
    }                                            \
    catch (const mnb::Error& e) {                \
        mnb::t_err = e.msg;                      \
        return e.code;                           \
    }                                            \
    catch (const std::exception& e) {            \
        mnb::t_err = e.what();                   \
        return MNB_EDEVICE;                      \
    }                                            \
    return MNB_OK;

extern "C" const char* mnb_last_error(void) { return mnb::t_err.c_str(); }

extern "C" int mnb_set_allocator(mnb_alloc_fn a, mnb_free_fn f, void* ctx) {
    if ((a == nullptr) != (f == nullptr)) {
        t_err = "allocator and free must both be set or both be NULL";
        return MNB_EINVAL;
    }
    g_alloc = a;
    g_free = f;
    g_ctx = ctx;
    return MNB_OK;
}
extern "C" int mnb_set_stream(void* s) {
    g_user_stream = (hipStream_t)s;
    return MNB_OK;
}

extern "C" int mnb_timer_begin(int kind, int node) {
    if (kind < MNB_T_FC_BACKSUB || kind > MNB_T_BOTTOM_WIN) {
        t_err = "bad timer kind";
        return MNB_EINVAL;
    }
    g_timer.kind = kind;
    g_timer.node = node;
    g_timer.used = 0;
    g_timer.flops = g_timer.bytes = 0;
    g_timer.running = true;
    return MNB_OK;
}

namespace {
int initial_variants() {
    int m = 0;
    if (getenv("MNB_BOTTOM_VALU")) m |= MNB_VAR_VALU_BOTTOM;
    if (getenv("MNB_NO_TAP_CONVT")) m |= MNB_VAR_NO_TAP_CONVT;
    if (getenv("MNB_NO_PAIR_CONV")) m |= MNB_VAR_NO_PAIR_CONV;
    if (getenv("MNB_NO_ROW_CONV")) m |= MNB_VAR_NO_ROW_CONV;
    if (getenv("MNB_NO_WIN_BOTTOM")) m |= MNB_VAR_NO_WINDOW;
    if (getenv("MNB_NO_FUSED_BOTTOM")) m |= MNB_VAR_NO_FUSED_BOTTOM;
    if (getenv("MNB_NO_PATCH")) m |= MNB_VAR_NO_PATCH;
    if (getenv("MNB_NO_CONE")) m |= MNB_VAR_NO_CONE;
    if (getenv("MNB_NO_FIRST_CONV")) m |= MNB_VAR_NO_FIRST_CONV;
    if (getenv("MNB_NO_WIN_CONV")) m |= MNB_VAR_NO_WIN_CONV;
    return m;
}
std::atomic<int> g_variants{initial_variants()};
}  // namespace

namespace mnb {
int kernel_variants() { return g_variants.load(std::memory_order_relaxed); }
}  // namespace mnb

extern "C" int mnb_set_kernel_variants(int mask) { return g_variants.exchange(mask); }
extern "C" int mnb_get_kernel_variants(void) { return g_variants.load(); }

extern "C" int mnb_timer_end(int64_t* launches, double* ms, double* flops, double* bytes) {
    API_BEGIN
    g_timer.running = false;
    sync();
    double tot = 0;
    for (size_t i = 0; i < g_timer.used; ++i) {
        float t = 0;
        MNB_HIP(hipEventElapsedTime(&t, g_timer.ev[i].first, g_timer.ev[i].second));
        tot += t;
    }
    if (launches) *launches = (int64_t)g_timer.used;
    if (ms) *ms = tot;
    if (flops) *flops = g_timer.flops;
    if (bytes) *bytes = g_timer.bytes;
    API_END
}

// =====================================================================================
// network
// =====================================================================================
mnb_net::~mnb_net() {
    for (void* p : owned) dfree(p);
}

// Device tables of a convolution Ci x Hi x Wi -> Co x Ho x Wo (k, s, p) with weights Wd / bd
// (host copy Wh): the forward gather table and the stride phases of the transposed one.
static void fill_conv_geom(mnb_net* net, ConvGeom& g, int Ci, int Hi, int Wi, int Co, int Ho, int Wo, int k, int s,
                           int p, const float* Wd, const float* bd, const std::vector<float>& Wh) {
    g.Ci = Ci; g.Hi = Hi; g.Wi = Wi;
    g.Co = Co; g.Ho = Ho; g.Wo = Wo;
    g.k = k; g.s = s; g.p = p;
    g.W = Wd; g.b = bd;
    // forward gather table and weights with K ordered (ky, kx, ci), input channel innermost
    std::vector<int2> ft((size_t)g.Ci * k * k);
    std::vector<float> wf((size_t)g.Co * g.Ci * k * k);
    for (int ky = 0; ky < k; ++ky)
        for (int kx = 0; kx < k; ++kx)
            for (int ci = 0; ci < g.Ci; ++ci) {
                const int kk2 = (ky * k + kx) * g.Ci + ci;
                ft[kk2] = make_int2(ci * g.Hi * g.Wi + ky * g.Wi + kx, (ky << 16) | kx);
                for (int co = 0; co < g.Co; ++co)
                    wf[(size_t)co * g.Ci * k * k + kk2] = Wh[(((size_t)co * g.Ci + ci) * k + ky) * k + kx];
            }
    g.fwd_ktab = upload(ft.data(), ft.size(), &net->owned);
    g.Wf = upload(wf.data(), wf.size(), &net->owned);
    g.Wg = nullptr;
    if (g.Ci % 16 == 0) {
        // the forward GEMM's K order: 16-channel groups outermost, so that the taps reading one
        // group's input region follow each other
        std::vector<float> wg(wf.size());
        for (int co = 0; co < g.Co; ++co)
            for (int cg = 0; cg < g.Ci / 16; ++cg)
                for (int t = 0; t < k * k; ++t)
                    for (int c = 0; c < 16; ++c)
                        wg[(size_t)co * g.Ci * k * k + ((size_t)cg * k * k + t) * 16 + c] =
                            wf[(size_t)co * g.Ci * k * k + (size_t)t * g.Ci + cg * 16 + c];
        g.Wg = upload(wg.data(), wg.size(), &net->owned);
    }
    g.Wt = nullptr;
    if (g.Ci % 8 == 0) {
        // the input-window kernel stages 8 input channels at a time: per group, per tap, per
        // channel a row of Co filter weights
        std::vector<float> wt(wf.size());
        for (int cg = 0; cg < g.Ci / 8; ++cg)
            for (int t = 0; t < k * k; ++t)
                for (int c = 0; c < 8; ++c)
                    for (int co = 0; co < g.Co; ++co)
                        wt[(((size_t)cg * k * k + t) * 8 + c) * g.Co + co] =
                            Wh[((size_t)co * g.Ci + cg * 8 + c) * k * k + t];
        g.Wt = upload(wt.data(), wt.size(), &net->owned);
    }
    // stride phases of the transposed convolution
    MNB_CHECK(s * s <= 16, MNB_EINVAL, "conv stride above 4 is not supported");
    g.n_phase = 0;
    for (int ry = 0; ry < s; ++ry)
        for (int rx = 0; rx < s; ++rx) {
            ConvPhase ph{};
            ph.rho_y = ry; ph.rho_x = rx;
            ph.Y0 = ((ry - g.p) % s + s) % s;
            ph.X0 = ((rx - g.p) % s + s) % s;
            ph.nY = ph.Y0 < g.Hi ? (g.Hi - ph.Y0 + s - 1) / s : 0;
            ph.nX = ph.X0 < g.Wi ? (g.Wi - ph.X0 + s - 1) / s : 0;
            ph.Ty = ry < k ? (k - ry + s - 1) / s : 0;
            ph.Tx = rx < k ? (k - rx + s - 1) / s : 0;
            ph.q0y = (ph.Y0 + g.p - ry) / s;
            ph.q0x = (ph.X0 + g.p - rx) / s;
            const int T = ph.Ty * ph.Tx;
            if (T > 0) {
                std::vector<float> wp((size_t)g.Co * T * g.Ci);
                std::vector<int2> kt((size_t)g.Co * T);
                // K ordered (ty, tx, co): output channel innermost
                for (int co = 0; co < g.Co; ++co)
                    for (int ty = 0; ty < ph.Ty; ++ty)
                        for (int tx = 0; tx < ph.Tx; ++tx) {
                            const int kk = (ty * ph.Tx + tx) * g.Co + co;
                            kt[kk] = make_int2(co * g.Ho * g.Wo - ty * g.Wo - tx, (ty << 16) | tx);
                            for (int ci = 0; ci < g.Ci; ++ci)
                                wp[(size_t)kk * g.Ci + ci] =
                                    Wh[(((size_t)co * g.Ci + ci) * k + (ry + s * ty)) * k + (rx + s * tx)];
                        }
                ph.Wp = upload(wp.data(), wp.size(), &net->owned);
                ph.ktab = upload(kt.data(), kt.size(), &net->owned);
                ph.Wpg = nullptr;
                if (g.Co % 16 == 0) {
                    // the transposed GEMM's K order: 16-channel groups outermost
                    std::vector<float> wg(wp.size());
                    for (int cg = 0; cg < g.Co / 16; ++cg)
                        for (int tt = 0; tt < T; ++tt)
                            for (int c = 0; c < 16; ++c)
                                for (int ci = 0; ci < g.Ci; ++ci)
                                    wg[(((size_t)cg * T + tt) * 16 + c) * g.Ci + ci] =
                                        wp[((size_t)tt * g.Co + cg * 16 + c) * g.Ci + ci];
                    ph.Wpg = upload(wg.data(), wg.size(), &net->owned);
                }
                ph.Wt = nullptr;
                if (g.Co % 8 == 0) {
                    // the phase as a stride-1 correlation for the input-window kernel: tap
                    // (Ty-1-ty, Tx-1-tx) reads coefficient (q0y + i - ty, q0x + j - tx)
                    std::vector<float> wt(wp.size());
                    for (int cg = 0; cg < g.Co / 8; ++cg)
                        for (int ty = 0; ty < ph.Ty; ++ty)
                            for (int tx = 0; tx < ph.Tx; ++tx)
                                for (int c = 0; c < 8; ++c)
                                    for (int ci = 0; ci < g.Ci; ++ci) {
                                        const int t = (ph.Ty - 1 - ty) * ph.Tx + (ph.Tx - 1 - tx);
                                        wt[(((size_t)cg * T + t) * 8 + c) * g.Ci + ci] =
                                            wp[((size_t)(ty * ph.Tx + tx) * g.Co + cg * 8 + c) * g.Ci + ci];
                                    }
                    ph.Wt = upload(wt.data(), wt.size(), &net->owned);
                }
            }
            g.ph[g.n_phase++] = ph;
        }
    g.Wt4 = nullptr;
    bool same = s == 2 && g.n_phase == 4 && g.Co % 8 == 0;
    for (int f = 0; same && f < 4; ++f)
        same = g.ph[f].Wt && g.ph[f].Ty > 0 && g.ph[f].Ty == g.ph[f].Tx && g.ph[f].Ty == g.ph[0].Ty &&
               g.ph[f].nY == g.ph[0].nY && g.ph[f].nX == g.ph[0].nX && g.ph[f].nY > 0 && g.ph[f].nX > 0;
    if (same) {
        // phase f's block of each 8-channel group follows phase f - 1's (the host copy of ph[f].Wt is
        // rebuilt here from the same weights)
        const int T = g.ph[0].Ty * g.ph[0].Tx;
        std::vector<float> w4((size_t)g.Co * 4 * T * g.Ci);
        for (int f = 0; f < 4; ++f) {
            const ConvPhase& ph = g.ph[f];
            for (int cg = 0; cg < g.Co / 8; ++cg)
                for (int ty = 0; ty < ph.Ty; ++ty)
                    for (int tx = 0; tx < ph.Tx; ++tx)
                        for (int c = 0; c < 8; ++c)
                            for (int ci = 0; ci < g.Ci; ++ci) {
                                const int t = (ph.Ty - 1 - ty) * ph.Tx + (ph.Tx - 1 - tx);
                                const int co = cg * 8 + c;
                                w4[((((size_t)cg * 4 + f) * T + t) * 8 + c) * g.Ci + ci] =
                                    Wh[(((size_t)co * g.Ci + ci) * k + (ph.rho_y + s * ty)) * k + (ph.rho_x + s * tx)];
                            }
        }
        g.Wt4 = upload(w4.data(), w4.size(), &net->owned);
    }
}

static void build_conv_geom(mnb_net* net, NetNode& nd, const std::vector<float>& Wh) {
    const NetNode& in = net->nodes[nd.src];
    fill_conv_geom(net, nd.geom, in.C, in.H, in.W, nd.C, nd.H, nd.W, nd.k, nd.stride, nd.pad, nd.Wd, nd.bd, Wh);
}

// Receptive-field plan of ReLU layer m (see PatchPlan): windows grow downwards, side
// P_in = (P_out - 1) s + k through a convolution k / s / p, origin stride S_in = S_out s and
// offset Q_in = Q_out s + p.  Used where the windows hold clearly fewer entries than the layers.
static PatchPlan make_patch_plan(mnb_net* net, int m, const std::map<int, std::vector<float>>& wh) {
    PatchPlan pp;
    if (m < 1) return pp;
    const int on = net->nodes[net->relus[m]].src;
    const NetNode& o = net->nodes[on];
    if (o.kind != MNB_CONV) return pp;
    const size_t nn = net->nodes.size();
    pp.g.assign(nn, PatchGeom{});
    pp.conv.assign(nn, ConvGeom{});
    pp.macs.assign(nn, 0.0);
    pp.top = o.src;
    int P = o.k, S = o.stride, Q = o.pad;
    long win = 0, dense = 0;
    int n = pp.top;
    while (true) {
        const NetNode& nd = net->nodes[n];
        pp.g[n] = PatchGeom{nd.C, nd.H, nd.W, P, S, Q, o.H * o.W, o.W};
        win += (long)nd.C * P * P;
        dense += nd.size;
        pp.max_width = std::max(pp.max_width, nd.C * P * P);
        if (n == 0) break;
        if (nd.kind == MNB_RELU) {
            n = nd.src;
        } else if (nd.kind == MNB_CONV) {
            const NetNode& in = net->nodes[nd.src];
            const int Pin = (P - 1) * nd.stride + nd.k;
            fill_conv_geom(net, pp.conv[n], in.C, Pin, Pin, nd.C, P, P, nd.k, nd.stride, 0, nd.Wd, nd.bd, wh.at(n));
            pp.macs[n] = (double)nd.C * in.C * nd.k * nd.k * P * P;
            P = Pin;
            S *= nd.stride;
            Q = Q * nd.stride + nd.pad;
            n = nd.src;
        } else {
            return PatchPlan{};
        }
    }
    // the pass buffers hold [M, max_width] and x* [M, d0]
    pp.ok = 2 * win <= dense && pp.max_width <= net->max_width && pp.width(0) <= net->d0;
    if (!pp.ok) return PatchPlan{};
    // forward cones, from the input up: a convolution k / s / p maps a cone [c, c + Pc) of its
    // input to the outputs y with y s - p <= c + Pc - 1 and y s - p + k - 1 >= c; its origin stays
    // affine in the objective position with the window's stride, so one convolution between
    // cones (padding c + p - y_min s) serves every row
    std::vector<int> chain;
    for (int m = pp.top; ; m = net->nodes[m].src) {
        chain.push_back(m);
        if (m == 0) break;
    }
    std::reverse(chain.begin(), chain.end());
    pp.fc.assign(nn, PatchGeom{});
    pp.fconv.assign(nn, ConvGeom{});
    pp.fmacs.assign(nn, 0.0);
    pp.fc[0] = pp.g[0];
    long cone = pp.fc[0].C * (long)pp.fc[0].P * pp.fc[0].P;
    bool ok = true;
    for (size_t t = 1; t < chain.size(); ++t) {
        const int m = chain[t];
        const NetNode& nd = net->nodes[m];
        const PatchGeom& in = pp.fc[nd.src];
        PatchGeom o = pp.g[m];
        if (nd.kind == MNB_CONV) {
            const int k = nd.k, s = nd.stride, p = nd.pad;
            const int c_in = -in.Q;   // cone origin for objective position 0
            auto fdiv = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
            const int y_min = -fdiv(-(c_in + p - k + 1), s);   // ceil
            const int y_max = fdiv(c_in + in.P - 1 + p, s);
            const int pad_v = c_in + p - y_min * s;
            o.Q = -y_min;
            o.P = y_max - y_min + 1;
            o.S = in.S / s;
            ok = ok && in.S % s == 0 && pad_v >= 0 && pad_v < k && o.P > 0;
            if (!ok) break;
            std::vector<float> zb(nd.C, 0.f);
            float* zbd = upload(zb.data(), zb.size(), &net->owned);
            fill_conv_geom(net, pp.fconv[m], net->nodes[nd.src].C, in.P, in.P, nd.C, o.P, o.P, k, s, pad_v, nd.Wd, zbd,
                           wh.at(m));
            pp.fmacs[m] = (double)nd.C * net->nodes[nd.src].C * k * k * o.P * o.P;
        } else {
            o.Q = in.Q;
            o.P = in.P;
            o.S = in.S;
        }
        // the cone holds the backward window of the node
        ok = ok && o.S == pp.g[m].S && -o.Q <= -pp.g[m].Q && -o.Q + o.P >= -pp.g[m].Q + pp.g[m].P;
        pp.fc[m] = o;
        cone += o.C * (long)o.P * o.P;
        ok = ok && o.C * (long)o.P * o.P <= net->max_width;
    }
    pp.cone_ok = ok && 3 * cone <= 2 * dense;
    return pp;
}

// Batch normalisation and average pooling are affine (Section 2.1 lists them among the layers the
// method covers): a batch normalisation y = gamma (x - mean) / sqrt(var + eps) + beta that follows a
// fully connected or convolutional node (its only consumer) is folded into that node's weights and
// bias, per output channel; an average pooling k x k / s / p becomes a convolution whose filter is
// 1/k^2 between equal channels and 0 elsewhere.  Later nodes are renumbered accordingly.
struct TranslatedNet {
    std::vector<mnb_layer> layers;
    std::vector<std::vector<float>> buffers;   // folded or generated weights and biases
};

static TranslatedNet translate_layers(const mnb_layer* L, int n) {
    TranslatedNet t;
    std::vector<int> map(n, -1), consumers(n, 0);
    std::vector<std::array<int, 3>> shp(n, std::array<int, 3>{0, 0, 0});   // output (C, H, W) of each node
    for (int i = 1; i < n; ++i) {
        MNB_CHECK(L[i].src >= 0 && L[i].src < i, MNB_EINVAL, "node " + std::to_string(i) + ": bad src");
        consumers[L[i].src]++;
        if (L[i].kind == MNB_ADD && L[i].src2 >= 0 && L[i].src2 < i) consumers[L[i].src2]++;
    }
    t.buffers.reserve(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        mnb_layer l = L[i];
        if (i == 0) {
            shp[0] = {l.out_chw[0], l.out_chw[1], l.out_chw[2]};
            map[0] = 0;
            t.layers.push_back(l);
            continue;
        }
        const auto& in = shp[l.src];
        switch (l.kind) {
            case MNB_BN: {
                mnb_layer& a = t.layers[map[l.src]];
                MNB_CHECK((a.kind == MNB_FC || a.kind == MNB_CONV) && consumers[l.src] == 1, MNB_EINVAL,
                          "batch normalisation must follow a fully connected or convolutional node, its only consumer");
                MNB_CHECK(l.W && l.eps >= 0.f && a.W && a.b, MNB_EINVAL,
                          "batch normalisation: need W = [gamma, beta, mean, var] per channel");
                const int C = in[0];
                const auto& ain = shp[L[l.src].src];
                const long per_c = a.kind == MNB_FC ? (long)ain[0] * ain[1] * ain[2] : (long)ain[0] * a.k * a.k;
                MNB_CHECK(C > 0 && per_c > 0, MNB_EINVAL, "batch normalisation: bad shape");
                // the folded node's weights and bias (copies: the caller's arrays are only read)
                std::vector<float> Wf(a.W, a.W + (size_t)C * per_c), bf(C);
                for (int c = 0; c < C; ++c) {
                    const double g = l.W[c], be = l.W[C + c], mu = l.W[2 * C + c], var = l.W[3 * C + c];
                    MNB_CHECK(var + (double)l.eps > 0.0, MNB_EINVAL, "batch normalisation: var + eps must be positive");
                    const double scale = g / std::sqrt(var + (double)l.eps);
                    for (long q = 0; q < per_c; ++q) Wf[c * per_c + q] = (float)((double)Wf[c * per_c + q] * scale);
                    bf[c] = (float)((double)a.b[c] * scale + (be - mu * scale));
                }
                t.buffers.push_back(std::move(Wf));
                a.W = t.buffers.back().data();
                t.buffers.push_back(std::move(bf));
                a.b = t.buffers.back().data();
                map[i] = map[l.src];
                shp[i] = in;
                continue;
            }
            case MNB_AVGPOOL: {
                const int C = in[0];
                MNB_CHECK(l.k > 0 && l.stride > 0 && l.pad >= 0 && C > 0, MNB_EINVAL, "average pooling: bad shape");
                std::vector<float> Wp((size_t)C * C * l.k * l.k, 0.f), bp(C, 0.f);
                const float v = 1.f / (float)(l.k * l.k);
                for (int c = 0; c < C; ++c)
                    for (int q = 0; q < l.k * l.k; ++q) Wp[((size_t)c * C + c) * l.k * l.k + q] = v;
                t.buffers.push_back(std::move(Wp));
                l.W = t.buffers.back().data();
                t.buffers.push_back(std::move(bp));
                l.b = t.buffers.back().data();
                l.kind = MNB_CONV;
                l.in_chw[0] = C;
                l.out_chw[0] = C;
                l.out_chw[1] = l.out_chw[2] = 0;   // derived from the input shape
                shp[i] = {C, (in[1] + 2 * l.pad - l.k) / l.stride + 1, (in[2] + 2 * l.pad - l.k) / l.stride + 1};
                break;
            }
            case MNB_FC:
                shp[i] = {l.out_chw[0], 1, 1};
                break;
            case MNB_CONV:
                shp[i] = {l.out_chw[0], l.k > 0 && l.stride > 0 ? (in[1] + 2 * l.pad - l.k) / l.stride + 1 : 0,
                          l.k > 0 && l.stride > 0 ? (in[2] + 2 * l.pad - l.k) / l.stride + 1 : 0};
                break;
            default:
                shp[i] = in;
                break;
        }
        l.src = map[l.src];
        if (l.kind == MNB_ADD) {
            MNB_CHECK(l.src2 >= 0 && l.src2 < i, MNB_EINVAL, "add: bad src2");
            l.src2 = map[l.src2];
        }
        map[i] = (int)t.layers.size();
        t.layers.push_back(l);
    }
    return t;
}

extern "C" int mnb_net_create(const mnb_layer* L_in, int n_in, mnb_net** out) {
    API_BEGIN
    MNB_CHECK(L_in && out && n_in >= 2, MNB_EINVAL, "need at least an input and one layer");
    MNB_CHECK(L_in[0].kind == MNB_INPUT, MNB_EINVAL, "node 0 must be MNB_INPUT");
    const TranslatedNet tn = translate_layers(L_in, n_in);
    const mnb_layer* L = tn.layers.data();
    const int n = (int)tn.layers.size();
    auto net = new mnb_net();
    try {
        std::map<int, std::vector<float>> conv_wh;   // host weights of the convolutions
        net->nodes.resize(n);
        for (int i = 0; i < n; ++i) {
            NetNode& nd = net->nodes[i];
            const mnb_layer& l = L[i];
            nd.kind = l.kind;
            nd.src = l.src;
            nd.src2 = l.src2;
            if (i == 0) {
                nd.C = l.out_chw[0]; nd.H = l.out_chw[1]; nd.W = l.out_chw[2];
                MNB_CHECK(nd.C > 0 && nd.H > 0 && nd.W > 0, MNB_EINVAL, "bad input shape");
            } else {
                MNB_CHECK(l.src >= 0 && l.src < i, MNB_EINVAL, "node " + std::to_string(i) + ": bad src");
                const NetNode& in = net->nodes[l.src];
                switch (l.kind) {
                    case MNB_FC: {
                        MNB_CHECK(l.out_chw[0] > 0 && l.W && l.b, MNB_EINVAL, "fc: need out_chw[0], W, b");
                        nd.C = l.out_chw[0]; nd.H = 1; nd.W = 1;
                        const int din = in.C * in.H * in.W;
                        nd.Wd = upload(l.W, (size_t)nd.C * din, &net->owned);
                        nd.bd = upload(l.b, (size_t)nd.C, &net->owned);
                        nd.macs_per_row = (double)nd.C * din;
                        break;
                    }
                    case MNB_CONV: {
                        MNB_CHECK(l.k > 0 && l.stride > 0 && l.pad >= 0 && l.W && l.b && l.out_chw[0] > 0,
                                  MNB_EINVAL, "conv: need k, stride, pad, W, b, out channels");
                        MNB_CHECK(in.C == l.in_chw[0] || l.in_chw[0] == 0, MNB_EINVAL, "conv: in channels");
                        nd.k = l.k; nd.stride = l.stride; nd.pad = l.pad;
                        nd.C = l.out_chw[0];
                        nd.H = (in.H + 2 * l.pad - l.k) / l.stride + 1;
                        nd.W = (in.W + 2 * l.pad - l.k) / l.stride + 1;
                        MNB_CHECK(nd.H > 0 && nd.W > 0, MNB_EINVAL, "conv: empty output");
                        if (l.out_chw[1]) MNB_CHECK(l.out_chw[1] == nd.H && l.out_chw[2] == nd.W, MNB_EINVAL,
                                                    "conv: output shape mismatch");
                        size_t nw = (size_t)nd.C * in.C * l.k * l.k;
                        std::vector<float> Wh(l.W, l.W + nw);
                        nd.Wd = upload(l.W, nw, &net->owned);
                        nd.bd = upload(l.b, (size_t)nd.C, &net->owned);
                        build_conv_geom(net, nd, Wh);
                        conv_wh[i] = std::move(Wh);
                        {
                            // nonzero multiply-adds per row: taps that do not fall on padding
                            double taps = 0;
                            for (int y = 0; y < nd.H; ++y)
                                for (int ky = 0; ky < l.k; ++ky) {
                                    int Y = y * l.stride - l.pad + ky;
                                    if (Y < 0 || Y >= in.H) continue;
                                    for (int x = 0; x < nd.W; ++x)
                                        for (int kx = 0; kx < l.k; ++kx) {
                                            int X = x * l.stride - l.pad + kx;
                                            if (X >= 0 && X < in.W) taps += 1;
                                        }
                                }
                            nd.macs_per_row = taps * nd.C * in.C;
                        }
                        break;
                    }
                    case MNB_RELU:
                        MNB_CHECK(in.kind == MNB_FC || in.kind == MNB_CONV || in.kind == MNB_ADD, MNB_EINVAL,
                                  "relu must follow fc, conv or add");
                        nd.C = in.C; nd.H = in.H; nd.W = in.W;
                        nd.relu_m = (int)net->relus.size();
                        net->relus.push_back(i);
                        break;
                    case MNB_ADD: {
                        MNB_CHECK(l.src2 >= 0 && l.src2 < i && l.src2 != l.src, MNB_EINVAL, "add: bad src2");
                        const NetNode& in2 = net->nodes[l.src2];
                        MNB_CHECK((in.kind == MNB_FC || in.kind == MNB_CONV) &&
                                      (in2.kind == MNB_FC || in2.kind == MNB_CONV),
                                  MNB_EINVAL, "add joins two affine nodes");
                        MNB_CHECK(in.C == in2.C && in.H == in2.H && in.W == in2.W, MNB_EINVAL,
                                  "add: shape mismatch");
                        MNB_CHECK(in.src != in2.src, MNB_EINVAL, "add: both operands read the same node");
                        nd.C = in.C; nd.H = in.H; nd.W = in.W;
                        break;
                    }
                    default:
                        throw Error{MNB_EINVAL, "unsupported node kind " + std::to_string(l.kind)};
                }
            }
            nd.size = nd.C * nd.H * nd.W;
            net->max_width = std::max(net->max_width, nd.size);
        }
        net->last = n - 1;
        MNB_CHECK(net->nodes[n - 1].kind == MNB_FC, MNB_EINVAL, "last node must be MNB_FC");
        // every affine/add node must have exactly one consumer (ReLU / ADD / the spec)
        std::vector<int> cons(n, 0);
        for (int i = 1; i < n; ++i) {
            cons[net->nodes[i].src]++;
            if (net->nodes[i].kind == MNB_ADD) cons[net->nodes[i].src2]++;
        }
        for (int i = 1; i < n - 1; ++i) {
            int kd = net->nodes[i].kind;
            if (kd == MNB_FC || kd == MNB_CONV || kd == MNB_ADD)
                MNB_CHECK(cons[i] == 1, MNB_EINVAL, "affine node " + std::to_string(i) + " needs exactly one consumer");
        }
        net->d0 = net->nodes[0].size;
        net->n_out = net->nodes[n - 1].size;
        int off = 0;
        for (int i : net->relus) {
            net->relu_d.push_back(net->nodes[i].size);
            net->relu_off.push_back(off);
            off += net->nodes[i].size;
            // effective bias of the node feeding this ReLU
            const NetNode& s = net->nodes[net->nodes[i].src];
            std::vector<float> bias(s.size, 0.f), tmp;
            auto add_bias = [&](const NetNode& a) {
                std::vector<float> bh(a.C);
                MNB_HIP(hipMemcpy(bh.data(), a.bd, a.C * sizeof(float), hipMemcpyDeviceToHost));
                for (int c = 0; c < a.C; ++c)
                    for (int q = 0; q < a.H * a.W; ++q) bias[c * a.H * a.W + q] += bh[c];
            };
            MNB_HIP(hipStreamSynchronize(stream()));
            if (s.kind == MNB_ADD) {
                add_bias(net->nodes[s.src]);
                add_bias(net->nodes[s.src2]);
            } else {
                add_bias(s);
            }
            net->relu_bias.push_back(upload(bias.data(), bias.size(), &net->owned));
        }
        net->total_d = off;
        MNB_CHECK(!net->relus.empty(), MNB_EINVAL, "network without ReLU layers");
        {
            const NetNode& r0 = net->nodes[net->relus[0]];
            const NetNode& a1 = net->nodes[r0.src];
            net->bottom_ok = a1.kind == MNB_CONV && a1.src == 0 &&
                             bottom_supported(r0.size, net->d0, a1.C * net->nodes[0].C * a1.k * a1.k);
            if (net->bottom_ok && net->relus.size() > 1) {
                const NetNode& on = net->nodes[net->nodes[net->relus[1]].src];
                net->win_ok = on.kind == MNB_CONV && on.src == net->relus[0] &&
                              win_supported(a1.C, net->nodes[0].C, a1.k, a1.stride, on.k, on.C, r0.size, net->d0);
            }
        }
        for (int m = 0; m < (int)net->relus.size(); ++m) net->patch.push_back(make_patch_plan(net, m, conv_wh));
        sync();
    } catch (...) {
        delete net;
        throw;
    }
    *out = net;
    API_END
}

extern "C" void mnb_net_destroy(mnb_net* net) {
    if (!net) return;
    try {
        sync();
    } catch (...) {
    }
    delete net;
}

extern "C" int mnb_net_info(const mnb_net* net, int* n_relu, int* relu_sizes, int* d_in, int* d_out) {
    API_BEGIN
    MNB_CHECK(net, MNB_EINVAL, "null net");
    if (n_relu) *n_relu = (int)net->relus.size();
    if (relu_sizes)
        for (size_t m = 0; m < net->relus.size(); ++m) relu_sizes[m] = net->relu_d[m];
    if (d_in) *d_in = net->d0;
    if (d_out) *d_out = net->n_out;
    API_END
}

// =====================================================================================
// problem
// =====================================================================================
mnb_problem::~mnb_problem() {
    for (void* p : owned) dfree(p);
}

static long pad16(long x) { return (x + 15) / 16 * 16; }

static void grow_queries(mnb_problem* pb) {
    int nc = std::max(4, pb->q_cap * 2);
    mnb_net* net = pb->net;
    const int S = pb->S, dl = net->nodes[net->nodes[net->last].src].size;
    auto regrow = [&](float*& p, long per) {
        float* np_ = (float*)dalloc(std::max<long>((long)nc * per * 4, 16));
        if (p) {
            MNB_HIP(hipMemcpyAsync(np_, p, (size_t)pb->q_cap * per * 4, hipMemcpyDeviceToDevice, stream()));
        }
        sync();
        if (p) {
            auto it = std::find(pb->owned.begin(), pb->owned.end(), (void*)p);
            if (it != pb->owned.end()) pb->owned.erase(it);
            dfree(p);
        }
        pb->owned.push_back(np_);
        p = np_;
    };
    auto regrow_i = [&](int*& p, long per) {
        float* f = (float*)p;
        regrow(f, per);
        p = (int*)f;
    };
    regrow(pb->lo, net->d0);
    regrow(pb->hi, net->d0);
    regrow(pb->Chat, (long)S * dl);
    regrow(pb->chat, S);
    regrow(pb->C, (long)S * net->n_out);
    regrow(pb->c0, S);
    if (pb->has_mnc) {
        for (int m = 0; m < pb->R; ++m) {
            auto& ml = pb->mnc[m];
            const int d = net->relu_d[m];
            regrow_i(ml.e_of, 1);
            regrow_i(ml.colptr, d + 1);
            regrow_i(ml.col_e, pb->nnz_cap);
            regrow(ml.col_P, pb->nnz_cap);
            regrow(ml.col_Ph, pb->nnz_cap);
            regrow_i(ml.rowptr, pb->e_cap + 1);
            regrow_i(ml.row_j, pb->nnz_cap);
            regrow(ml.row_P, pb->nnz_cap);
            regrow(ml.row_Ph, pb->nnz_cap);
            regrow(ml.p, pb->e_cap);
        }
    }
    pb->q_cap = nc;
}

extern "C" int mnb_problem_create(const mnb_net* net, int n_spec, int64_t capacity, int max_mnc,
                                  mnb_problem** out) {
    API_BEGIN
    MNB_CHECK(net && out && n_spec > 0 && capacity > 0 && max_mnc >= 0, MNB_EINVAL, "bad problem arguments");
    auto pb = new mnb_problem();
    try {
        pb->net = (mnb_net*)net;
        pb->S = n_spec;
        pb->cap = capacity;
        pb->R = (int)net->relus.size();
        pb->n_sets = 2 * pb->R - 1;
        pb->e_cap = max_mnc;
        pb->has_mnc = max_mnc > 0;
        pb->nnz_cap = 4 * max_mnc;
        pb->ld_state = pad16(net->total_d);
        pb->ld_param = pb->ld_state;
        pb->ld_gamma = pad16((long)pb->R * max_mnc);
        const long cap = capacity;
        auto A = [&](size_t bytes) {
            void* p = dalloc(std::max<size_t>(bytes, 16));
            pb->owned.push_back(p);
            return p;
        };
        pb->l = (float*)A(cap * pb->ld_state * 4);
        pb->u = (float*)A(cap * pb->ld_state * 4);
        pb->S_ = (int8_t*)A(cap * pb->ld_state);
        pb->alpha = (float*)A(cap * pb->n_sets * pb->ld_param * 4);
        pb->beta = (float*)A(cap * pb->n_sets * pb->ld_param * 4);
        pb->gamma = (float*)A(cap * pb->n_sets * pb->ld_gamma * 4);
        pb->qid = (int32_t*)A(cap * 4);
        pb->lb = (float*)A(cap * pb->S * 4);
        pb->recompute_from.assign(cap, pb->R);
        pb->slot_query.assign(cap, -1);
        pb->used.assign(cap, 0);
        for (int64_t s = cap - 1; s >= 0; --s) pb->free_list.push_back(s);
        pb->mnc.resize(pb->R);
        grow_queries(pb);
    } catch (...) {
        delete pb;
        throw;
    }
    *out = pb;
    API_END
}

extern "C" void mnb_problem_destroy(mnb_problem* pb) {
    if (!pb) return;
    try {
        sync();
    } catch (...) {
    }
    delete pb;
}

// Per-slot device bytes of a problem (bounds, split signs, parameter sets, query index, reported lb).
size_t mnb::problem_slot_bytes(const mnb_problem* pb) {
    return (size_t)pb->ld_state * 9 + (size_t)pb->n_sets * (pb->ld_param * 8 + pb->ld_gamma * 4) + 4 + (size_t)pb->S * 4;
}

// Grow the slot pool to `capacity` slots: every per-slot array is reallocated and copied (on the
// stream, then synchronised); ids stay valid.  Callers hold the problem's lock or own it alone.
void mnb::problem_grow(mnb_problem* pb, int64_t capacity) {
    if (capacity <= pb->cap) return;
    const long oc = pb->cap, nc = capacity;
    hipStream_t st = stream();
    auto regrow = [&](void*& p, size_t per_slot) {
        void* np_ = dalloc(std::max<size_t>(nc * per_slot, 16));
        MNB_HIP(hipMemcpyAsync(np_, p, oc * per_slot, hipMemcpyDeviceToDevice, st));
        sync();
        auto it = std::find(pb->owned.begin(), pb->owned.end(), p);
        if (it != pb->owned.end()) *it = np_;
        dfree(p);
        p = np_;
    };
    auto grow_f = [&](float*& p, size_t per) {
        void* v = p;
        regrow(v, per * 4);
        p = (float*)v;
    };
    grow_f(pb->l, pb->ld_state);
    grow_f(pb->u, pb->ld_state);
    {
        void* v = pb->S_;
        regrow(v, pb->ld_state);
        pb->S_ = (int8_t*)v;
    }
    grow_f(pb->alpha, (size_t)pb->n_sets * pb->ld_param);
    grow_f(pb->beta, (size_t)pb->n_sets * pb->ld_param);
    grow_f(pb->gamma, (size_t)pb->n_sets * pb->ld_gamma);
    {
        void* v = pb->qid;
        regrow(v, 4);
        pb->qid = (int32_t*)v;
    }
    grow_f(pb->lb, pb->S);
    pb->recompute_from.resize(nc, pb->R);
    pb->slot_query.resize(nc, -1);
    pb->used.resize(nc, 0);
    // new slots handed out after the existing free ones, lowest index first
    std::vector<int64_t> fresh;
    for (int64_t s = nc - 1; s >= oc; --s) fresh.push_back(s);
    pb->free_list.insert(pb->free_list.begin(), fresh.begin(), fresh.end());
    pb->cap = nc;
}

static int64_t alloc_slot(mnb_problem* pb) {
    if (pb->free_list.empty()) throw Error{MNB_ENOMEM, "problem capacity exhausted"};
    int64_t s = pb->free_list.back();
    pb->free_list.pop_back();
    pb->used[s] = 1;
    pb->n_used++;
    return s;
}
static void check_id(mnb_problem* pb, int64_t id) {
    MNB_CHECK(id >= 0 && id < pb->cap && pb->used[id], MNB_EINVAL, "invalid subproblem id " + std::to_string(id));
}

extern "C" int mnb_release(mnb_problem* pb, const int64_t* ids, int n) {
    API_BEGIN
    MNB_CHECK(pb && (ids || n == 0), MNB_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(pb->mu);
    for (int i = 0; i < n; ++i) check_id(pb, ids[i]);
    for (int i = 0; i < n; ++i) {
        if (!pb->used[ids[i]]) continue;   // duplicate within the call
        pb->used[ids[i]] = 0;
        pb->free_list.push_back(ids[i]);
        pb->n_used--;
    }
    API_END
}

extern "C" int mnb_problem_usage(const mnb_problem* pb, int64_t* used, int64_t* capacity) {
    API_BEGIN
    MNB_CHECK(pb, MNB_EINVAL, "null problem");
    if (used) *used = pb->n_used;
    if (capacity) *capacity = pb->cap;
    API_END
}

// =====================================================================================
// passes
// =====================================================================================
namespace {

struct PassChunk {
    // row chunks of the fused bottom kernel (built on first use)
    std::vector<int> bchunk_inst, bchunk_r0, bchunk_r1, bchunk_first, bchunk_last;
    int* bchunk_d = nullptr;
    // per-window row lists of the window bottom kernel (built on first use)
    int* win_ptr_d = nullptr;
    WinEnt* win_ent_d = nullptr;
    int M = 0;                  // rows
    const RowDesc* rows = nullptr;   // device, chunk-relative row order
    std::vector<InstDesc> inst;      // host, rows relative to the chunk
    InstDesc* inst_d = nullptr;
    int obj_layer = -1;         // ReLU layer of the objective, -1: spec rows
    // octahedral rows (multi-neuron constraint generation): row 26 g + s is sum_t s_t e_{grp[g][t]}
    // on the input of ReLU layer obj_layer, for the 26 directions s; groups [M / 26][3] on the device
    const int32_t* oct_groups = nullptr;
    // receptive-field rows (nullable): windows of each row's deviation from its instance's
    // shared row
    const PatchPlan* pp = nullptr;
    bool cone = false;                // the adjoint runs on forward cones
    int inst_base = 0;                // pass-wide index of the chunk's first instance
    // the shared rows, one per instance (descriptors built on first use)
    RowDesc* sh_rows_d = nullptr;
    InstDesc* sh_inst_d = nullptr;
    bool zero_rows = false;           // rows are the zero objective (a chunk of shared rows)
    // cone adjoint: instance i's rows run in kRowSlice-row slices, slice z of it writing partial
    // gradient sums at slot zoff[i] + z (nz_max slices at most per instance, nz_total in all)
    int* zoff_d = nullptr;
    int nz_total = 0, nz_max = 0;
};

// Row width of a chunk's coefficients on node n.
static int node_width(const mnb_net* net, const PassChunk& ch, int n) {
    return ch.pp ? ch.pp->width(n) : net->nodes[n].size;
}

// A pool of [M, max_width] coefficient buffers with reference counts.
struct BufPool {
    std::vector<float*> bufs;
    std::vector<int> ref;
    float* acquire() {
        for (size_t i = 0; i < bufs.size(); ++i)
            if (ref[i] == 0) {
                ref[i] = 1;
                return bufs[i];
            }
        throw Error{MNB_EDEVICE, "coefficient buffer pool exhausted"};
    }
    void retain(float* p) {
        for (size_t i = 0; i < bufs.size(); ++i)
            if (bufs[i] == p) ref[i]++;
    }
    void release(float* p) {
        for (size_t i = 0; i < bufs.size(); ++i)
            if (bufs[i] == p) ref[i]--;
    }
};

struct PassCtx {
    mnb_problem* pb;
    const int32_t* slots_d;   // local b -> global slot
    float* c;                 // [M]
    float* cpart; int ldcp;
    int ncp = 0;
    std::map<int, float*> ap; // relu node -> a' rows [M, d] (nullable)
    float* G0 = nullptr;      // [M, d0]
    uint8_t* xbits = nullptr; // [M, d0]
    // gamma projections per relu layer: v, vhat [n_inst, d], gp [n_inst]
    std::map<int, float*> v, vh, gp;
    // adjoint checkpoints (ckpt_stride > 1): the live coefficient rows copied before every
    // stride-th ReLU of the pass (top first), with the partial-constant column at that point
    int ckpt_stride = 1;
    struct Ckpt {
        int node;
        int col;
        std::map<int, float*> coef;
    };
    std::vector<Ckpt> ckpts;
    Workspace* ws = nullptr;
    // rows +-e_j on a fully connected layer's output not materialised: the first fold of the
    // pass reads sign W[j] (fold_W, fold_b: weights and objective bias; consumed by that fold)
    const float* fold_W = nullptr;
    const float* fold_b = nullptr;
    const RowDesc* fold_rows = nullptr;
    // receptive-field rows: a' deviation windows per relu node [M, window]; the shared rows'
    // relaxation table per relu node [n_inst, d] (read by the deviation folds, or written by the
    // folds of the shared rows)
    std::map<int, float*> apw;
    std::map<int, float4*> rt_in, rt_out;
};

static int fold_cols(int d) { return cdiv(d, 256) * 4; }

// Rounding margin of a reported (spec-row) bound: lb is lowered by 2^-20 (sum_j |a_j| max(|lo_j|,
// |hi_j|) + |c|), which covers the FP32 rounding of the concretisation where the bound is exact.
// Intermediate bounds are concretised without it.
constexpr float kSpecMargin = 9.5367431640625e-07f;

// Total partial-constant columns of a pass whose rows start at node `top`.
static int pass_cols(const mnb_net* net, int top, const PatchPlan* pp = nullptr) {
    int cols = 0;
    for (int i : net->relus)
        if (i <= top) cols += fold_cols(pp ? pp->width(i) : net->nodes[i].size);
    return std::max(cols, 1);
}

static int pass_top(const mnb_net* net, int obj_layer) {
    if (obj_layer < 0) return net->nodes[net->last].src;
    const NetNode& o = net->nodes[net->nodes[net->relus[obj_layer]].src];
    if (o.kind == MNB_ADD) return std::max(net->nodes[o.src].src, net->nodes[o.src2].src);
    return o.src;
}

// Highest node a chunk's rows are on: octahedral rows start on the ReLU input node itself.
static int chunk_top(const mnb_net* net, const PassChunk& ch) {
    if (ch.oct_groups) return net->nodes[net->relus[ch.obj_layer]].src;
    return pass_top(net, ch.obj_layer);
}

// Back-substitute a chunk of rows from its objective down to the input (Eq. 2 and
// Eq. 5 per node, in reverse topological order) and leave the input coefficients
// in the returned buffer.
// Process nodes (to, from] of a pass in reverse topological order (Eq. 2 / Eq. 5 per
// node).  With record_ckpt and a checkpoint stride > 1 the live coefficient rows are
// copied before every stride-th ReLU (counting from the top of the pass).
static void walk_backsub(PassCtx& cx, const PassChunk& ch, BufPool& pool, std::map<int, float*>& coef, int from,
                         int to, bool store_ap, int& col, bool record_ckpt) {
    mnb_problem* pb = cx.pb;
    mnb_net* net = pb->net;
    hipStream_t st = stream();
    const int M = ch.M;
    int relu_seen = 0;
    for (int n = from; n > to; --n) {
        auto it = coef.find(n);
        if (it == coef.end()) continue;
        if (record_ckpt && cx.ckpt_stride > 1 && net->nodes[n].kind == MNB_RELU) {
            if (relu_seen % cx.ckpt_stride == 0) {
                PassCtx::Ckpt ck;
                ck.node = n;
                ck.col = col;
                for (auto& kv : coef) {
                    const size_t cnt = (size_t)M * net->nodes[kv.first].size;
                    float* cp = cx.ws->get<float>("ck" + std::to_string(cx.ckpts.size()) + "_" + std::to_string(kv.first),
                                                  cnt);
                    MNB_HIP(hipMemcpyAsync(cp, kv.second, cnt * sizeof(float), hipMemcpyDeviceToDevice, st));
                    ck.coef[kv.first] = cp;
                }
                cx.ckpts.push_back(ck);
            }
            ++relu_seen;
        }
        float* a = it->second;
        coef.erase(it);
        const NetNode& nd = net->nodes[n];
        switch (nd.kind) {
            case MNB_FC:
            case MNB_CONV: {
                const int dst = nd.src;
                bool acc = coef.count(dst) > 0;
                float* out = acc ? coef[dst] : pool.acquire();
                {
                    TimerScope ts(nd.kind == MNB_FC ? MNB_T_FC_BACKSUB : MNB_T_CONV_BACKSUB, n,
                                  2.0 * M * (ch.pp ? ch.pp->macs[n] : nd.macs_per_row),
                                  4.0 * M * (node_width(net, ch, n) + node_width(net, ch, dst) * (acc ? 2 : 1)));
                    if (nd.kind == MNB_FC)
                        launch_fc_backsub(a, nd.Wd, out, M, nd.size, net->nodes[dst].size, acc, st);
                    else
                        launch_conv_backsub(ch.pp ? ch.pp->conv[n] : nd.geom, a, out, M, acc, st);
                }
                coef[dst] = out;
                pool.release(a);
                break;
            }
            case MNB_RELU: {
                const int m = nd.relu_m;
                FoldArgs fa{};
                fa.A = a;
                fa.Ap = store_ap ? (ch.pp ? cx.apw.at(n) : cx.ap.at(n)) : nullptr;
                fa.cpart = cx.cpart; fa.ldcp = cx.ldcp; fa.col_off = col;
                fa.inst = ch.inst_d; fa.n_inst = (int)ch.inst.size();
                fa.slots = cx.slots_d;
                fa.M = M; fa.d = nd.size;
                fa.l = pb->l + net->relu_off[m]; fa.u = pb->u + net->relu_off[m];
                fa.S = pb->S_ + net->relu_off[m]; fa.ld_state = pb->ld_state;
                fa.alpha = pb->alpha + net->relu_off[m]; fa.beta = pb->beta + net->relu_off[m];
                fa.ld_param = pb->ld_param; fa.n_sets = pb->n_sets;
                fa.v = cx.v.count(m) ? cx.v[m] : nullptr;
                fa.vhat = cx.vh.count(m) ? cx.vh[m] : nullptr;
                fa.bias = net->relu_bias[m];
                if (cx.fold_W) {
                    fa.Wsrc = cx.fold_W;
                    fa.rows = cx.fold_rows;
                    fa.c = cx.c;
                    fa.bias_obj = cx.fold_b;
                    cx.fold_W = nullptr;
                }
                {
                    TimerScope ts(MNB_T_FOLD, n, 0.0, (double)M * node_width(net, ch, n) * (store_ap ? 12 : 8));
                    fa.rt_out = cx.rt_out.count(n) ? cx.rt_out[n] : nullptr;
                    if (ch.pp) {
                        fa.rt_in = cx.rt_in.at(n);
                        launch_relu_fold_patch(fa, ch.pp->g[n], ch.rows, ch.inst_base, st);
                    } else
                        launch_relu_fold(fa, st, cx.gp.count(m) ? cx.gp[m] : nullptr);
                }
                col += fold_cols(node_width(net, ch, n));
                MNB_CHECK(!coef.count(nd.src), MNB_EDEVICE, "relu input reached twice");
                coef[nd.src] = a;
                break;
            }
            case MNB_ADD: {
                coef[nd.src] = a;
                MNB_CHECK(!coef.count(nd.src2), MNB_EDEVICE, "add operand reached twice");
                coef[nd.src2] = a;
                pool.retain(a);
                break;
            }
            default:
                throw Error{MNB_EDEVICE, "unexpected node in back-substitution"};
        }
    }
}

static float* run_backsub(PassCtx& cx, const PassChunk& ch, BufPool& pool, bool store_ap, int stop = 0) {
    mnb_problem* pb = cx.pb;
    mnb_net* net = pb->net;
    hipStream_t st = stream();
    const int M = ch.M;
    std::map<int, float*> coef;
    int top;
    if (ch.oct_groups) {
        top = chunk_top(net, ch);
        float* A = pool.acquire();
        launch_init_oct(ch.oct_groups, M / 26, net->nodes[top].size, net->relu_bias[ch.obj_layer], A, cx.c, st);
        coef[top] = A;
    } else if (ch.zero_rows) {
        // the zero objective (shared rows of receptive-field passes): coefficient and constant 0
        top = pass_top(net, ch.obj_layer);
        float* A = pool.acquire();
        launch_fill(A, (long)M * net->nodes[top].size, 0.f, st);
        launch_fill(cx.c, M, 0.f, st);
        coef[top] = A;
    } else if (ch.pp) {
        // receptive-field rows: sign W[co] on the objective convolution's input window
        const NetNode& o = net->nodes[net->nodes[net->relus[ch.obj_layer]].src];
        top = ch.pp->top;
        float* A = pool.acquire();
        launch_init_conv_patch(ch.rows, M, o.Wd, net->relu_bias[ch.obj_layer], net->nodes[top].C * o.k * o.k,
                               o.H * o.W, A, cx.c, st);
        coef[top] = A;
    } else if (ch.obj_layer < 0) {
        top = net->nodes[net->last].src;
        float* A = pool.acquire();
        const int d = net->nodes[top].size;
        launch_init_spec(ch.rows, M, cx.slots_d, pb->qid, pb->Chat, pb->chat, pb->S, d, A, cx.c, st);
        coef[top] = A;
    } else {
        const int ri = net->relus[ch.obj_layer];
        const int on = net->nodes[ri].src;
        const NetNode& o = net->nodes[on];
        const float* be = net->relu_bias[ch.obj_layer];
        auto init_aff = [&](int n, bool write_c) {
            const NetNode& a = net->nodes[n];
            float* A = pool.acquire();
            if (a.kind == MNB_FC)
                launch_init_fc(ch.rows, M, a.Wd, be, net->nodes[a.src].size, A, cx.c, write_c, st);
            else
                launch_init_conv(ch.rows, M, a.geom, be, A, cx.c, write_c, st);
            MNB_CHECK(!coef.count(a.src), MNB_EINVAL, "objective operands share a producer");
            coef[a.src] = A;
        };
        if (o.kind == MNB_ADD) {
            init_aff(o.src, true);
            init_aff(o.src2, false);
        } else if (o.kind == MNB_FC && net->nodes[o.src].kind == MNB_RELU && cx.ckpt_stride <= 1) {
            // the rows are sign W[j] on the FC input: the ReLU fold that comes first reads them
            // from W (no checkpoint copies this coefficient before that fold)
            coef[o.src] = pool.acquire();
            cx.fold_W = o.Wd;
            cx.fold_b = be;
            cx.fold_rows = ch.rows;
        } else {
            init_aff(on, true);
        }
        top = pass_top(net, ch.obj_layer);
    }
    int col = 0;
    walk_backsub(cx, ch, pool, coef, top, stop, store_ap, col, true);
    cx.ncp = col;
    MNB_CHECK(coef.size() == 1 && coef.count(stop), MNB_EDEVICE, "back-substitution did not reach its stop node");
    return coef[stop];
}

// Adjoint of a pass: push x* forward through every row's relaxation and reduce
// the parameter gradients of each instance.
static void run_adjoint(PassCtx& cx, const PassChunk& ch, BufPool& pool, float* g_alpha, float* g_beta,
                        float* g_gamma, float* gs_hat, float* gs_out, int start = 0, float* g_start = nullptr) {
    mnb_problem* pb = cx.pb;
    mnb_net* net = pb->net;
    hipStream_t st = stream();
    const int M = ch.M;
    const int top = chunk_top(net, ch);
    const int n_inst = (int)ch.inst.size();
    std::vector<float*> g(net->nodes.size(), nullptr);
    std::vector<int> uses(net->nodes.size(), 0);
    for (int n = start + 1; n <= top; ++n) {
        uses[net->nodes[n].src]++;
        if (net->nodes[n].kind == MNB_ADD) uses[net->nodes[n].src2]++;
    }
    g[start] = start == 0 ? cx.G0 : g_start;
    auto done_with = [&](int n) {
        if (--uses[n] == 0 && n != 0) pool.release(g[n]);
    };
    // checkpointed mode: rebuild a' of one segment (between two checkpoints) from its
    // checkpoint just before the forward pass reaches it; only that segment's a' is live
    std::set<int> ready;
    auto recompute_segment = [&](int n) {
        int s = -1;
        for (int k = 0; k < (int)cx.ckpts.size(); ++k)
            if (cx.ckpts[k].node >= n) s = k;
        MNB_CHECK(s >= 0, MNB_EDEVICE, "no checkpoint above ReLU node " + std::to_string(n));
        const PassCtx::Ckpt& ck = cx.ckpts[s];
        const int lower = s + 1 < (int)cx.ckpts.size() ? cx.ckpts[s + 1].node : start;
        std::map<int, float*> coef;
        for (auto& kv : ck.coef) {
            float* b = pool.acquire();
            MNB_HIP(hipMemcpyAsync(b, kv.second, (size_t)M * net->nodes[kv.first].size * sizeof(float),
                                   hipMemcpyDeviceToDevice, st));
            coef[kv.first] = b;
        }
        int k = 0;
        for (int i = ck.node; i > lower; --i)
            if (net->nodes[i].kind == MNB_RELU) {
                cx.ap[i] = cx.ws->get<float>("apseg" + std::to_string(k++), (size_t)M * net->max_width);
                ready.insert(i);
            }
        int col = ck.col;
        walk_backsub(cx, ch, pool, coef, ck.node, lower, true, col, false);
        std::set<float*> live;
        for (auto& kv : coef) live.insert(kv.second);
        for (auto& kv : coef) pool.release(kv.second);
    };
    for (int n = start + 1; n <= top; ++n) {
        const NetNode& nd = net->nodes[n];
        switch (nd.kind) {
            case MNB_FC:
            case MNB_CONV: {
                float* out = pool.acquire();
                {
                    TimerScope ts(nd.kind == MNB_FC ? MNB_T_FC_FORWARD : MNB_T_CONV_FORWARD, n,
                                  2.0 * M * nd.macs_per_row, 4.0 * M * (nd.size + net->nodes[nd.src].size));
                    if (nd.kind == MNB_FC)
                        launch_fc_forward(g[nd.src], nd.Wd, nd.bd, out, M, net->nodes[nd.src].size, nd.size, false,
                                          st);
                    else
                        launch_conv_forward(nd.geom, g[nd.src], out, M, false, st);
                }
                g[n] = out;
                done_with(nd.src);
                break;
            }
            case MNB_ADD: {
                float* out = g[nd.src];
                launch_add2(g[nd.src], g[nd.src2], out, (long)M * nd.size, st);
                g[n] = out;
                pool.retain(out);
                done_with(nd.src);
                done_with(nd.src2);
                break;
            }
            case MNB_RELU: {
                const int m = nd.relu_m;
                if (cx.ckpt_stride > 1 && !ready.count(n)) recompute_segment(n);
                float* G = g[nd.src];
                RelaxArgs ra{};
                ra.G = G;
                ra.Ap = cx.ap.at(n);
                ra.inst = ch.inst_d; ra.n_inst = n_inst;
                ra.slots = cx.slots_d;
                ra.M = M; ra.d = nd.size;
                ra.l = pb->l + net->relu_off[m]; ra.u = pb->u + net->relu_off[m];
                ra.S = pb->S_ + net->relu_off[m]; ra.ld_state = pb->ld_state;
                ra.alpha = pb->alpha + net->relu_off[m]; ra.ld_param = pb->ld_param; ra.n_sets = pb->n_sets;
                ra.d_alpha = g_alpha; ra.d_beta = g_beta; ra.ldg = pb->ld_param; ra.goff = net->relu_off[m];
                const bool mnc = pb->has_mnc;
                ra.gsum_hat = mnc ? gs_hat : nullptr;
                ra.gsum_out = mnc ? gs_out : nullptr;
                {
                    TimerScope ts(MNB_T_RELAX, n, 0.0, 12.0 * M * nd.size);
                    launch_relu_relax(ra, st);
                }
                if (mnc) {
                    auto& ml = pb->mnc[m];
                    GammaArgs ga{};
                    ga.inst = ch.inst_d; ga.n_inst = n_inst; ga.qid = pb->qid;
                    ga.gamma = pb->gamma; ga.ld_gamma = pb->ld_gamma; ga.n_sets = pb->n_sets;
                    ga.goff = m * pb->e_cap;
                    ga.d = nd.size; ga.e_cap = pb->e_cap; ga.nnz_cap = pb->nnz_cap;
                    ga.e_of = ml.e_of; ga.colptr = ml.colptr; ga.col_e = ml.col_e; ga.col_P = ml.col_P;
                    ga.col_Ph = ml.col_Ph; ga.rowptr = ml.rowptr; ga.row_j = ml.row_j; ga.row_P = ml.row_P;
                    ga.row_Ph = ml.row_Ph; ga.p = ml.p;
                    launch_gamma_grad(ga, gs_hat, gs_out, g_gamma, pb->ld_gamma, st);
                }
                g[n] = G;   // relaxed in place
                if (uses[nd.src] == 1) {
                    uses[nd.src] = 0;
                } else {
                    pool.retain(G);
                    done_with(nd.src);
                }
                break;
            }
            default:
                throw Error{MNB_EDEVICE, "unexpected node in adjoint"};
        }
    }
    for (int n = std::max(start, 1); n <= top; ++n)
        if (uses[n] > 0 && g[n]) {
            uses[n] = 0;
            pool.release(g[n]);
        }
}

// gamma projections v = P^T gamma, vhat = Phat^T gamma, gp = gamma . p for every
// ReLU layer below the objective of a chunk.
static void gamma_projections(PassCtx& cx, const PassChunk& ch, Workspace& ws, const std::string& tag) {
    mnb_problem* pb = cx.pb;
    if (!pb->has_mnc) return;
    mnb_net* net = pb->net;
    const int top = chunk_top(net, ch);
    const int n_inst = (int)ch.inst.size();
    for (int m = 0; m < pb->R; ++m) {
        const int ri = net->relus[m];
        if (ri > top) break;
        const int d = net->relu_d[m];
        float* v = ws.get<float>(tag + "v" + std::to_string(m), (size_t)n_inst * d);
        float* vh = ws.get<float>(tag + "vh" + std::to_string(m), (size_t)n_inst * d);
        float* gp = ws.get<float>(tag + "gp" + std::to_string(m), (size_t)n_inst);
        auto& ml = pb->mnc[m];
        GammaArgs ga{};
        ga.inst = ch.inst_d; ga.n_inst = n_inst; ga.qid = pb->qid;
        ga.gamma = pb->gamma; ga.ld_gamma = pb->ld_gamma; ga.n_sets = pb->n_sets; ga.goff = m * pb->e_cap;
        ga.d = d; ga.e_cap = pb->e_cap; ga.nnz_cap = pb->nnz_cap;
        ga.e_of = ml.e_of; ga.colptr = ml.colptr; ga.col_e = ml.col_e; ga.col_P = ml.col_P; ga.col_Ph = ml.col_Ph;
        ga.rowptr = ml.rowptr; ga.row_j = ml.row_j; ga.row_P = ml.row_P; ga.row_Ph = ml.row_Ph; ga.p = ml.p;
        ga.v = v; ga.vhat = vh; ga.gp = gp;
        launch_gamma_proj(ga, stream());
        cx.v[m] = v;
        cx.vh[m] = vh;
        cx.gp[m] = gp;
    }
}

// Device workspace needed by a chunk of M rows of a pass with the given top node.
static size_t chunk_bytes(const mnb_net* net, int top, long M, int n_inst, bool adjoint,
                          const PatchPlan* pp = nullptr) {
    size_t b = 0;
    b += 3 * (size_t)M * net->max_width * 4;            // coefficient / forward buffers
    b += (size_t)M * (pass_cols(net, top) + 1) * 4;     // c + partials
    b += (size_t)M * net->d0 * 5;                       // x* floats + bits
    if (adjoint)
        for (int i : net->relus)
            if (i <= top) b += (size_t)M * net->nodes[i].size * 4;   // a'
    b += (size_t)n_inst * net->total_d * 4 * 4;         // gradients / sums
    if (pp) {
        // shared rows (one per instance, whole layers, with their relaxation tables and forward
        // values) and the deviation windows of a'
        b += (size_t)n_inst * (3 * (size_t)net->max_width + 7 * (size_t)net->total_d + net->d0 + pass_cols(net, top) + 2) * 4;
        if (adjoint) {
            for (int i : net->relus)
                if (i <= top) b += (size_t)M * pp->width(i) * 4;
            // partial gradient sums of the cone relaxation's row slices
            b += (size_t)(M / kRowSlice + n_inst) * 3 * net->max_width * 4;
        }
    }
    return b;
}

}  // namespace

// =====================================================================================
// evaluation of chunks (shared by bound_init and bound_optimize)
// =====================================================================================
namespace {

struct ChunkIO {
    // spec-row outputs (mode 1)
    float* lb_rows = nullptr;     // [M]
    float* best = nullptr;        // [M]
    uint8_t* improved = nullptr;  // [M]
    uint8_t* best_bits = nullptr; // [M, d0]
};

// Evaluate one chunk (back-substitution + concretisation), optionally followed
// by its adjoint and a projected Adam step.
struct Evaluator {
    mnb_problem* pb;
    const int32_t* slots_d;
    Workspace& ws;
    Evaluator(mnb_problem* p, const int32_t* s) : pb(p), slots_d(s), ws(p->ws) {}
    Evaluator(mnb_problem* p, const int32_t* s, Workspace& w) : pb(p), slots_d(s), ws(w) {}

    BufPool make_pool(int M, int nbuf, int width) {
        BufPool pool;
        for (int i = 0; i < nbuf; ++i) {
            pool.bufs.push_back(ws.get<float>("pool" + std::to_string(i), (size_t)M * width));
            pool.ref.push_back(0);
        }
        return pool;
    }

    // The shared rows of a receptive-field chunk: for every instance the back-substitution of the
    // zero objective with the instance's parameters (whole layers): a' per ReLU node, the input
    // coefficients U0, their x* and bound.
    struct SharedRows {
        std::map<int, float*> ap;
        std::map<int, float4*> rt;    // relaxation table per ReLU node
        std::map<int, float*> ghat;   // forward values at each ReLU's input (cone adjoint)
        float* U0 = nullptr;
        float* x0 = nullptr;
        float* lb = nullptr;
        BufPool pool;
    };
    void shared_rows(const PassChunk& ch, const PassCtx& rcx, SharedRows& sh) {
        mnb_net* net = pb->net;
        hipStream_t st = stream();
        const int n = (int)ch.inst.size();
        auto& c = const_cast<PassChunk&>(ch);
        if (!ch.sh_rows_d) {
            std::vector<RowDesc> rd(n);
            std::vector<InstDesc> id(n);
            for (int i = 0; i < n; ++i) {
                rd[i] = RowDesc{ch.inst[i].b, ch.inst_base + i, 0, 0};
                id[i] = ch.inst[i];
                id[i].r0 = i;
                id[i].r1 = i + 1;
            }
            const std::string tg = std::to_string((long)ch.inst_d);
            c.sh_rows_d = ws.get<RowDesc>("shr" + tg, n);
            c.sh_inst_d = ws.get<InstDesc>("shi" + tg, n);
            h2d(c.sh_rows_d, rd.data(), n * sizeof(RowDesc));
            h2d(c.sh_inst_d, id.data(), n * sizeof(InstDesc));
        }
        PassChunk sc;
        sc.M = n;
        sc.rows = ch.sh_rows_d;
        sc.inst = ch.inst;
        for (int i = 0; i < n; ++i) {
            sc.inst[i].r0 = i;
            sc.inst[i].r1 = i + 1;
        }
        sc.inst_d = ch.sh_inst_d;
        sc.obj_layer = ch.obj_layer;
        sc.zero_rows = true;
        const int top = chunk_top(net, sc);
        PassCtx cs{};
        cs.pb = pb;
        cs.slots_d = slots_d;
        cs.c = ws.get<float>("sh_c", n);
        cs.ldcp = pass_cols(net, top);
        cs.cpart = ws.get<float>("sh_cpart", (size_t)n * cs.ldcp);
        cs.ws = &ws;
        cs.v = rcx.v;
        cs.vh = rcx.vh;
        cs.gp = rcx.gp;
        for (int i : net->relus)
            if (i <= top) {
                cs.ap[i] = ws.get<float>("sh_ap" + std::to_string(i), (size_t)n * net->nodes[i].size);
                cs.rt_out[i] = ws.get<float4>("sh_rt" + std::to_string(i), (size_t)n * net->nodes[i].size);
            }
        for (int i = 0; i < 3; ++i) {
            sh.pool.bufs.push_back(ws.get<float>("sh_pool" + std::to_string(i), (size_t)n * net->max_width));
            sh.pool.ref.push_back(0);
        }
        sh.U0 = run_backsub(cs, sc, sh.pool, true);
        sh.ap = cs.ap;
        sh.rt = cs.rt_out;
        sh.x0 = ws.get<float>("sh_x0", (size_t)n * net->d0);
        sh.lb = ws.get<float>("sh_lb", n);
        ConcArgs ca{};
        ca.mode = 2;
        ca.A = sh.U0; ca.c = cs.c; ca.cpart = cs.cpart; ca.ldcp = cs.ldcp; ca.ncp = cs.ncp;
        ca.rows = sc.rows; ca.slots = slots_d; ca.qid = pb->qid; ca.lo = pb->lo; ca.hi = pb->hi;
        ca.M = n; ca.d0 = net->d0;
        ca.G0 = sh.x0;
        ca.lb_out = sh.lb;
        launch_concretize(ca, st);
    }

    // Forward values of the shared rows (their x* through their own relaxation, whole layers),
    // kept at every ReLU input for the cone adjoint.
    void shared_forward(const PassChunk& ch, SharedRows& sh) {
        mnb_net* net = pb->net;
        hipStream_t st = stream();
        const int n = (int)ch.inst.size();
        const int top = chunk_top(net, ch);
        const float* gp = sh.x0;
        for (int m = 1; m <= top; ++m) {
            const NetNode& nd = net->nodes[m];
            if (nd.kind == MNB_CONV) {
                float* out = ws.get<float>("sh_f" + std::to_string(m), (size_t)n * nd.size);
                {
                    TimerScope ts(MNB_T_CONV_FORWARD, m, 2.0 * n * nd.macs_per_row,
                                  4.0 * n * (nd.size + net->nodes[nd.src].size));
                    launch_conv_forward(nd.geom, gp, out, n, false, st);
                }
                gp = out;
            } else if (nd.kind == MNB_RELU) {
                const int r = nd.relu_m;
                sh.ghat[m] = const_cast<float*>(gp);
                float* gs = ws.get<float>("sh_g" + std::to_string(m), (size_t)n * nd.size);
                RelaxArgs ra{};
                ra.inst = ch.inst_d; ra.n_inst = n; ra.d = nd.size;
                ra.l = pb->l + net->relu_off[r]; ra.u = pb->u + net->relu_off[r];
                ra.S = pb->S_ + net->relu_off[r]; ra.ld_state = pb->ld_state;
                ra.alpha = pb->alpha + net->relu_off[r]; ra.ld_param = pb->ld_param; ra.n_sets = pb->n_sets;
                launch_relax_shared(ra, sh.ap.at(m), gp, gs, st);
                gp = gs;
            } else {
                throw Error{MNB_EDEVICE, "unexpected node in a receptive-field pass"};
            }
        }
    }

    // Adjoint of receptive-field rows on forward cones: the rows' x* deviation (G0, cone of the
    // input) is pushed up through the convolutions between cones; each ReLU relaxes the rows'
    // deviations and reduces the instance's gradients with the shared rows' terms.
    void adjoint_cone(PassCtx& cx, const PassChunk& ch, BufPool& pool, const SharedRows& sh, float* g_alpha,
                      float* g_beta, float* g_gamma, float* gs_hat, float* gs_out) {
        mnb_net* net = pb->net;
        hipStream_t st = stream();
        const int M = ch.M, n_inst = (int)ch.inst.size();
        const int top = chunk_top(net, ch);
        const PatchPlan& pp = *ch.pp;
        float* g = cx.G0;
        bool clipped = false;   // g's cone entries outside the node hold 0
        for (int m = 1; m <= top; ++m) {
            const NetNode& nd = net->nodes[m];
            if (nd.kind == MNB_CONV) {
                float* out = pool.acquire();
                {
                    TimerScope ts(MNB_T_CONV_FORWARD, m, 2.0 * M * pp.fmacs[m],
                                  4.0 * M * (pp.cone_width(m) + pp.cone_width(nd.src)));
                    const PatchGeom& fc = pp.fc[m];
                    const ConeClip clip{ch.rows, nd.H, nd.W, fc.S, fc.Q, fc.HWobj, fc.Wobj};
                    launch_conv_forward(pp.fconv[m], g, out, M, false, st, &clip);
                }
                if (g != cx.G0) pool.release(g);
                g = out;
                clipped = true;
            } else {
                if (!clipped) launch_cone_zero(pp.fc[m], ch.rows, M, g, st);
                const int r = nd.relu_m;
                RelaxArgs ra{};
                ra.inst = ch.inst_d; ra.n_inst = n_inst; ra.slots = cx.slots_d;
                ra.M = M; ra.d = nd.size;
                ra.l = pb->l + net->relu_off[r]; ra.u = pb->u + net->relu_off[r];
                ra.S = pb->S_ + net->relu_off[r]; ra.ld_state = pb->ld_state;
                ra.alpha = pb->alpha + net->relu_off[r]; ra.ld_param = pb->ld_param; ra.n_sets = pb->n_sets;
                ra.d_alpha = g_alpha; ra.d_beta = g_beta; ra.ldg = pb->ld_param; ra.goff = net->relu_off[r];
                ra.gsum_hat = pb->has_mnc ? gs_hat : nullptr;
                ra.gsum_out = pb->has_mnc ? gs_out : nullptr;
                {
                    TimerScope ts(MNB_T_RELAX, m, 0.0, 8.0 * M * pp.cone_width(m) + 4.0 * M * pp.width(m));
                    MNB_CHECK(ch.zoff_d != nullptr, MNB_EDEVICE, "row slices missing");
                    ra.zoff = ch.zoff_d; ra.n_slices = ch.nz_max;
                    ra.part = ws.get<float>("relax_part", (size_t)ch.nz_total * 3 * nd.size);
                    launch_relax_cone(ra, pp.g[m], pp.fc[m], ch.rows, sh.ap.at(m), sh.ghat.at(m), cx.apw.at(m), g,
                                      st);
                }
                if (pb->has_mnc) {
                    auto& ml = pb->mnc[r];
                    GammaArgs ga{};
                    ga.inst = ch.inst_d; ga.n_inst = n_inst; ga.qid = pb->qid;
                    ga.gamma = pb->gamma; ga.ld_gamma = pb->ld_gamma; ga.n_sets = pb->n_sets;
                    ga.goff = r * pb->e_cap;
                    ga.d = nd.size; ga.e_cap = pb->e_cap; ga.nnz_cap = pb->nnz_cap;
                    ga.e_of = ml.e_of; ga.colptr = ml.colptr; ga.col_e = ml.col_e; ga.col_P = ml.col_P;
                    ga.col_Ph = ml.col_Ph; ga.rowptr = ml.rowptr; ga.row_j = ml.row_j; ga.row_P = ml.row_P;
                    ga.row_Ph = ml.row_Ph; ga.p = ml.p;
                    launch_gamma_grad(ga, gs_hat, gs_out, g_gamma, pb->ld_gamma, st);
                }
            }
        }
        if (g != cx.G0) pool.release(g);
    }

    bool no_write = false;   // concretise intermediate rows without touching l/u, skip Adam
    int ckpt_stride = 1;     // adjoint checkpoint stride over ReLU layers (1: keep every a')
    float *g_alpha_last = nullptr, *g_beta_last = nullptr, *g_gamma_last = nullptr;
    void eval(const PassChunk& ch, bool adjoint, bool keep_ap, const ChunkIO& io, const mnb_opt_cfg* cfg,
              float* m_alpha, float* v_alpha, float* m_beta, float* v_beta, float* m_gamma, float* v_gamma, int t) {
        mnb_net* net = pb->net;
        hipStream_t st = stream();
        const int M = ch.M;
        if (M == 0) return;
        const int top = chunk_top(net, ch);
        PassCtx cx{};
        cx.pb = pb;
        cx.slots_d = slots_d;
        cx.c = ws.get<float>("c", M);
        cx.ldcp = pass_cols(net, top, ch.pp);
        cx.cpart = ws.get<float>("cpart", (size_t)M * cx.ldcp);
        cx.G0 = ws.get<float>("G0", (size_t)M * net->d0);
        cx.ws = &ws;
        // receptive-field rows keep the deviation windows of a' (no checkpoints)
        cx.ckpt_stride = (adjoint && !keep_ap && ckpt_stride > 1 && !ch.pp) ? ckpt_stride : 1;
        const bool want_ap = (adjoint || keep_ap) && cx.ckpt_stride == 1;
        if (want_ap)
            for (int i : net->relus)
                if (i <= top) {
                    if (!ch.cone)
                        cx.ap[i] = ws.get<float>("ap" + std::to_string(i), (size_t)M * net->nodes[i].size);
                    if (ch.pp) cx.apw[i] = ws.get<float>("apw" + std::to_string(i), (size_t)M * ch.pp->width(i));
                }
        if (ch.obj_layer < 0) cx.xbits = ws.get<uint8_t>("xbits", (size_t)M * net->d0);
        gamma_projections(cx, ch, ws, "gproj");
        BufPool pool = make_pool(M, cx.ckpt_stride > 1 ? 6 : 3, net->max_width);
        // receptive-field rows: first the shared row of every instance (whole layers)
        SharedRows sh;
        if (ch.pp) {
            shared_rows(ch, cx, sh);
            cx.rt_in = sh.rt;
            if (adjoint && ch.cone) shared_forward(ch, sh);
        }
        const int r0n = net->relus[0];
        const bool fused = net->bottom_ok && ch.obj_layer != 0 && !ch.pp &&
                           !(kernel_variants() & MNB_VAR_NO_FUSED_BOTTOM);
        float* g_bottom = nullptr;
        if (fused) {
            // back-substitute down to the output of ReLU layer 0 (or build the rows there) and
            // finish the pass, and the first part of its adjoint, in the fused bottom kernel
            const NetNode& a1 = net->nodes[net->nodes[r0n].src];
            BottomArgs ba{};
            float* A1 = nullptr;
            bool src1 = false;
            if (ch.obj_layer == 1 && !ch.oct_groups) {
                const NetNode& on = net->nodes[net->nodes[net->relus[1]].src];
                src1 = on.kind == MNB_CONV && on.src == r0n;
                if (src1) {
                    ba.Wobj = on.Wd; ba.bias_obj = net->relu_bias[1];
                    ba.oCi = on.geom.Ci; ba.oHi = on.geom.Hi; ba.oWi = on.geom.Wi;
                    ba.oCo = on.C; ba.oHo = on.H; ba.oWo = on.W; ba.ok = on.k; ba.os = on.stride; ba.op = on.pad;
                }
            }
            if (!src1) {
                A1 = run_backsub(cx, ch, pool, want_ap, r0n);
            } else {
                cx.ncp = 0;
            }
            ba.src_mode = src1 ? 1 : 0;
            ba.A = A1; ba.c = cx.c; ba.cpart = cx.cpart; ba.ldcp = cx.ldcp; ba.ncp = cx.ncp;
            ba.rows = ch.rows; ba.inst = ch.inst_d; ba.slots = slots_d; ba.qid = pb->qid;
            ba.M = M; ba.d1 = net->relu_d[0]; ba.d0 = net->d0;
            ba.Ci = a1.geom.Ci; ba.Hi = a1.geom.Hi; ba.Wi = a1.geom.Wi;
            ba.Co = a1.C; ba.Ho = a1.H; ba.Wo = a1.W; ba.k = a1.k; ba.s = a1.stride; ba.p = a1.pad;
            ba.W1 = a1.Wd; ba.b1 = a1.bd; ba.bias1 = net->relu_bias[0];
            ba.l = pb->l; ba.u = pb->u; ba.S = pb->S_; ba.ld_state = pb->ld_state;
            ba.alpha = pb->alpha; ba.beta = pb->beta; ba.ld_param = pb->ld_param; ba.n_sets = pb->n_sets;
            ba.v = cx.v.count(0) ? cx.v[0] : nullptr;
            ba.vhat = cx.vh.count(0) ? cx.vh[0] : nullptr;
            ba.gp = cx.gp.count(0) ? cx.gp[0] : nullptr;
            ba.lo = pb->lo; ba.hi = pb->hi;
            if (ch.obj_layer < 0) {
                ba.mode = 1;
                ba.lb_out = io.lb_rows; ba.best = io.best; ba.improved = io.improved; ba.xbits = cx.xbits;
            } else if (no_write) {
                ba.mode = 2;
                ba.lb_out = io.lb_rows;
            } else {
                ba.mode = 0;
                ba.lw = pb->l; ba.uw = pb->u; ba.state_off_obj = net->relu_off[ch.obj_layer];
            }
            ba.margin = ch.obj_layer < 0 ? kSpecMargin : 0.f;
            ba.adjoint = adjoint;
            const int top = chunk_top(net, ch);
            if (adjoint && top > r0n) g_bottom = pool.acquire();
            ba.Gout = g_bottom;
            ba.Ap_out = keep_ap ? cx.ap.at(r0n) : nullptr;
            if (adjoint || keep_ap) {
                const int n_inst = (int)ch.inst.size();
                ba.d_alpha = ws.get<float>("g_alpha", (size_t)n_inst * pb->ld_param);
                ba.d_beta = ws.get<float>("g_beta", (size_t)n_inst * pb->ld_param);
                ba.ldg = pb->ld_param;
                if (pb->has_mnc) {
                    ba.gsum_hat = ws.get<float>("gs_hat0", (size_t)n_inst * net->max_width);
                    ba.gsum_out = ws.get<float>("gs_out0", (size_t)n_inst * net->max_width);
                }
            }
            if (src1 && net->win_ok && !pb->has_mnc && !keep_ap && !(kernel_variants() & MNB_VAR_NO_WINDOW)) {
                // window-sparse rows: one workgroup per (instance, window position)
                const NetNode& on = net->nodes[net->nodes[net->relus[1]].src];
                const int n_inst = (int)ch.inst.size();
                WinArgs wa{};
                wa.mode = ba.mode;
                wa.rows = ch.rows; wa.inst = ch.inst_d; wa.qid = pb->qid;
                wa.d1 = net->relu_d[0]; wa.d0 = net->d0;
                wa.Ci = a1.geom.Ci; wa.Hi = a1.geom.Hi; wa.Wi = a1.geom.Wi;
                wa.C1 = a1.C; wa.Ho = a1.H; wa.Wo = a1.W; wa.k = a1.k; wa.s = a1.stride; wa.p = a1.pad;
                wa.W1 = a1.Wd; wa.b1 = a1.bd;
                wa.oCi = on.geom.Ci; wa.oHi = on.geom.Hi; wa.oWi = on.geom.Wi;
                wa.oCo = on.C; wa.oHo = on.H; wa.oWo = on.W; wa.ok = on.k; wa.os = on.stride; wa.op = on.pad;
                wa.Wobj = on.Wd; wa.bobj = net->relu_bias[1];
                wa.l = pb->l; wa.u = pb->u; wa.S = pb->S_; wa.ld_state = pb->ld_state;
                wa.alpha = pb->alpha; wa.beta = pb->beta; wa.ld_param = pb->ld_param; wa.n_sets = pb->n_sets;
                wa.lo = pb->lo; wa.hi = pb->hi;
                wa.lw = ba.lw; wa.uw = ba.uw; wa.state_off_obj = ba.state_off_obj;
                wa.lb_out = ba.lb_out;
                wa.adjoint = adjoint;
                wa.asplit = ws.get<float>("w_as", (size_t)n_inst * net->d0);
                const bool lists = ch.win_ptr_d == nullptr;
                if (lists) {
                    auto& c = const_cast<PassChunk&>(ch);
                    const std::string tg = std::to_string((long)ch.inst_d);
                    c.win_ptr_d = ws.get<int>("wptr" + tg, (size_t)n_inst * (on.H * on.W + 1));
                    c.win_ent_d = ws.get<WinEnt>("went" + tg, (size_t)M);
                }
                wa.win_ptr = ch.win_ptr_d;
                wa.win_ent = ch.win_ent_d;
                wa.scal = ws.get<float>("w_sc", (size_t)n_inst * 4);
                const int nwin = on.H * on.W, E = a1.C * on.k * on.k;
                const int IH = (on.k - 1) * a1.stride + a1.k;
                if (adjoint) {
                    wa.part_a = ws.get<float>("w_pa", (size_t)n_inst * nwin * E);
                    wa.part_x = ws.get<float>("w_px", (size_t)n_inst * nwin * a1.geom.Ci * IH * IH);
                    wa.part_n = ws.get<int>("w_pn", (size_t)n_inst * nwin);
                    wa.d_alpha = ba.d_alpha; wa.d_beta = ba.d_beta; wa.ldg = ba.ldg;
                }
                if (lists) launch_win_rows(wa, n_inst, st);
                {
                    const double macs = (double)on.k * on.k * a1.C * a1.geom.Ci * a1.k * a1.k;
                    TimerScope ts(MNB_T_BOTTOM_WIN, r0n, 2.0 * M * (adjoint ? 2.0 : 1.0) * macs, 0.0);
                    launch_bottom_win(wa, n_inst, st);
                }
                launch_bottom_win_reduce(wa, n_inst, st);
            } else {
                // fixed 16-row chunks per instance (independent of the rest of the batch)
                const int n_inst = (int)ch.inst.size();
                if (ch.bchunk_inst.empty()) {
                    auto& c = const_cast<PassChunk&>(ch);
                    for (int i = 0; i < n_inst; ++i) {
                        c.bchunk_first.push_back((int)c.bchunk_inst.size());
                        for (int r = ch.inst[i].r0; r < ch.inst[i].r1; r += BOTTOM_CHUNK_ROWS) {
                            c.bchunk_inst.push_back(i);
                            c.bchunk_r0.push_back(r);
                            c.bchunk_r1.push_back(std::min(r + BOTTOM_CHUNK_ROWS, ch.inst[i].r1));
                        }
                        c.bchunk_last.push_back((int)c.bchunk_inst.size());
                    }
                    const std::string tg = "bch" + std::to_string((long)ch.inst_d);
                    const int nc = (int)c.bchunk_inst.size();
                    int* dv = ws.get<int>(tg, (size_t)3 * nc + 2 * n_inst + 4);
                    std::vector<int> hv;
                    hv.insert(hv.end(), c.bchunk_inst.begin(), c.bchunk_inst.end());
                    hv.insert(hv.end(), c.bchunk_r0.begin(), c.bchunk_r0.end());
                    hv.insert(hv.end(), c.bchunk_r1.begin(), c.bchunk_r1.end());
                    hv.insert(hv.end(), c.bchunk_first.begin(), c.bchunk_first.end());
                    hv.insert(hv.end(), c.bchunk_last.begin(), c.bchunk_last.end());
                    h2d(dv, hv.data(), hv.size() * 4);
                    c.bchunk_d = dv;
                }
                const int nc = (int)ch.bchunk_inst.size();
                ba.cinst = ch.bchunk_d;
                ba.cr0 = ch.bchunk_d + nc;
                ba.cr1 = ch.bchunk_d + 2 * nc;
                ba.ichunk0 = ch.bchunk_d + 3 * nc;
                ba.ichunk1 = ch.bchunk_d + 3 * nc + n_inst;
                ba.n_chunk = nc;
                if (adjoint) ba.part = ws.get<float>("bpart", (size_t)nc * (2 * net->relu_d[0] + net->d0));
                {
                    // algorithmic bytes: coefficient rows read (unless built from the filter),
                    // gradient rows and a' rows written, x* bits written
                    const double rowb = (double)M * net->relu_d[0] * 4.0;
                    TimerScope ts(MNB_T_BOTTOM, r0n, 2.0 * M * (adjoint ? 2.0 : 1.0) * a1.macs_per_row,
                                  rowb * ((src1 ? 0.0 : 1.0) + (ba.Gout ? 1.0 : 0.0) + (ba.Ap_out ? 1.0 : 0.0)) +
                                      (ba.xbits ? (double)M * net->d0 : 0.0));
                    launch_bottom(ba, n_inst, st);
                }
                launch_bottom_reduce(ba, n_inst, st);
            }
            if (A1) pool.release(A1);
            if (ch.obj_layer < 0 && io.best_bits)
                launch_keep_best_x(cx.xbits, io.best_bits, io.improved, M, net->d0, st);
        } else {
        float* A0 = run_backsub(cx, ch, pool, want_ap);
        ConcArgs ca{};
        ca.A = A0; ca.c = cx.c; ca.cpart = cx.cpart; ca.ldcp = cx.ldcp; ca.ncp = cx.ncp;
        ca.rows = ch.rows; ca.slots = slots_d; ca.qid = pb->qid; ca.lo = pb->lo; ca.hi = pb->hi;
        ca.M = M; ca.d0 = net->d0;
        ca.G0 = adjoint ? cx.G0 : nullptr;
        if (ch.pp) {
            // whole rows for the adjoint: x* and a' of the shared row plus each row's window
            ca.pg = ch.pp->g[0];
            ca.ush0 = sh.U0; ca.lbs = sh.lb; ca.inst_base = ch.inst_base;
            ca.g0_dev = ch.cone;
            if (adjoint && !ch.cone) {
                launch_patch_expand(sh.x0, nullptr, ch.rows, M, ch.inst_base, ch.pp->g[0], cx.G0, st);
                for (int i : net->relus)
                    if (i <= top)
                        launch_patch_expand(sh.ap.at(i), cx.apw.at(i), ch.rows, M, ch.inst_base, ch.pp->g[i],
                                            cx.ap.at(i), st);
            }
        }
        ca.margin = ch.obj_layer < 0 ? kSpecMargin : 0.f;
        if (ch.obj_layer < 0) {
            ca.mode = 1;
            ca.xbits = cx.xbits;
            ca.lb_out = io.lb_rows; ca.best = io.best; ca.improved = io.improved;
        } else if (no_write) {
            ca.mode = 2;
            ca.lb_out = io.lb_rows;
        } else {
            ca.mode = 0;
            ca.l = pb->l; ca.u = pb->u; ca.ld_state = pb->ld_state;
            ca.state_off = net->relu_off[ch.obj_layer];
        }
        {
            TimerScope ts(MNB_T_CONCRETIZE, 0, 0.0,
                          (double)M * node_width(net, ch, 0) * (4 + (ca.G0 ? 4 : 0) + (ca.xbits ? 1 : 0)));
            launch_concretize(ca, st);
        }
        pool.release(A0);
        if (sh.pool.bufs.size() && sh.U0) sh.pool.release(sh.U0);
        if (ch.obj_layer < 0 && io.best_bits)
            launch_keep_best_x(cx.xbits, io.best_bits, io.improved, M, net->d0, st);
        }
        if (keep_ap) last_ap = cx.ap;
        if (!adjoint) return;
        const int n_inst = (int)ch.inst.size();
        float* g_alpha = ws.get<float>("g_alpha", (size_t)n_inst * pb->ld_param);
        float* g_beta = ws.get<float>("g_beta", (size_t)n_inst * pb->ld_param);
        float* g_gamma = pb->has_mnc ? ws.get<float>("g_gamma", (size_t)n_inst * pb->ld_gamma) : nullptr;
        float* gs_hat = pb->has_mnc ? ws.get<float>("gs_hat", (size_t)n_inst * net->max_width) : nullptr;
        float* gs_out = pb->has_mnc ? ws.get<float>("gs_out", (size_t)n_inst * net->max_width) : nullptr;
        if (pb->has_mnc) launch_fill(g_gamma, (long)n_inst * pb->ld_gamma, 0.f, st);
        if (fused) {
            if (pb->has_mnc) {
                // gamma gradient of ReLU layer 0 from the bottom kernel's column sums
                auto& ml = pb->mnc[0];
                GammaArgs ga{};
                ga.inst = ch.inst_d; ga.n_inst = n_inst; ga.qid = pb->qid;
                ga.gamma = pb->gamma; ga.ld_gamma = pb->ld_gamma; ga.n_sets = pb->n_sets; ga.goff = 0;
                ga.d = net->relu_d[0]; ga.e_cap = pb->e_cap; ga.nnz_cap = pb->nnz_cap;
                ga.e_of = ml.e_of; ga.colptr = ml.colptr; ga.col_e = ml.col_e; ga.col_P = ml.col_P;
                ga.col_Ph = ml.col_Ph; ga.rowptr = ml.rowptr; ga.row_j = ml.row_j; ga.row_P = ml.row_P;
                ga.row_Ph = ml.row_Ph; ga.p = ml.p;
                launch_gamma_grad(ga, ws.get<float>("gs_hat0", (size_t)n_inst * net->max_width),
                                  ws.get<float>("gs_out0", (size_t)n_inst * net->max_width), g_gamma, pb->ld_gamma, st);
            }
            if (g_bottom) run_adjoint(cx, ch, pool, g_alpha, g_beta, g_gamma, gs_hat, gs_out, r0n, g_bottom);
        } else if (ch.pp && ch.cone) {
            adjoint_cone(cx, ch, pool, sh, g_alpha, g_beta, g_gamma, gs_hat, gs_out);
        } else {
            run_adjoint(cx, ch, pool, g_alpha, g_beta, g_gamma, gs_hat, gs_out);
        }
        g_alpha_last = g_alpha;
        g_beta_last = g_beta;
        g_gamma_last = g_gamma;
        if (no_write) return;
        // projected Adam ascent on every instance's set
        AdamArgs aa{};
        aa.inst = ch.inst_d; aa.n_inst = n_inst;
        aa.alpha = pb->alpha; aa.beta = pb->beta; aa.ld_param = pb->ld_param; aa.n_sets = pb->n_sets;
        aa.m_alpha = m_alpha; aa.v_alpha = v_alpha; aa.m_beta = m_beta; aa.v_beta = v_beta;
        aa.g_alpha = g_alpha; aa.g_beta = g_beta; aa.ldg = pb->ld_param;
        const int obj = ch.obj_layer < 0 ? pb->R : ch.obj_layer;
        aa.n_ab = obj < pb->R ? net->relu_off[obj] : net->total_d;
        aa.l = pb->l; aa.u = pb->u; aa.S = pb->S_; aa.ld_state = pb->ld_state;
        aa.gamma = pb->has_mnc ? pb->gamma : nullptr;
        aa.m_gamma = m_gamma; aa.v_gamma = v_gamma; aa.g_gamma = g_gamma; aa.ld_gamma = pb->ld_gamma;
        aa.n_gamma = pb->has_mnc ? obj * pb->e_cap : 0;
        aa.lr = cfg->lr; aa.b1 = cfg->beta1; aa.b2 = cfg->beta2; aa.eps = cfg->eps;
        aa.bc1 = 1.f - powf(cfg->beta1, (float)(t + 1));
        aa.bc2 = 1.f - powf(cfg->beta2, (float)(t + 1));
        launch_adam(aa, st);
    }
    std::map<int, float*> last_ap;
};

}  // namespace

#include "engine_calls.inc"
