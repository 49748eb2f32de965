// Windowed implicit-GEMM convolution: the forward product of the adjoint (x* through a
// convolutional layer) and, one stride phase at a time or four phases per workgroup, the
// transposed convolution of back-substitution (Eq. 2).
//
// One workgroup owns one row and a tile of BM output positions of the layer (whole output rows
// where they fit).  For 8 input channels at a time it stages the input window those positions
// read, and the filters of the channels, once into LDS; the MFMA then reads both operands
// straight from there, so every input element is fetched from memory once per workgroup
// instead of once per filter tap that reads it.  The filters are the MFMA's A operand and the
// window the B operand, which puts the output positions along the lanes of the result: a
// fragment's stores are 16 consecutive positions of one channel.
//
// Window layout (per staged channel, plane stride PL): window row wy = input row
// S y_first - p + wy; window column j = input column + CO, split into S phases of WS columns
// (column j at phase j % S, index j / S), so that the 16 lanes of a fragment, which hold
// consecutive output columns x, read consecutive words for every tap even at stride 2.  Padding
// is zero-filled once per workgroup; only in-range input elements are staged.
//
// An output element sums its products in an order set by the layer alone (8-channel groups,
// then taps, then channel quads), whatever the batch and tile: a row's result does not depend
// on the rows around it.
#include "kernels.h"
#include "../../include/mnbab.h"

namespace mnb {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

constexpr int CG = 8;          // input channels per LDS stage
constexpr int NLD4 = 6;        // float4 window loads per thread and stage, at most
constexpr int NLD1 = 12;       // scalar window loads per thread and stage, at most
constexpr size_t WIN_LDS_MAX = 64 * 1024;

struct ConvWinArgs {
    const float* G; float* C; const float* Wt; const float* bias;   // bias nullable
    long ldG, ldC;
    int Hi, Wi, Co, Ho, Wo, p, px, n_groups;   // p / px: padding of rows / columns
    int mtiles, acc;
    int CO, RS, WS, PL;
    // output position (y, x) of channel n at n*out_ns + (out_y0 + out_s y)*out_rs + out_x0 + out_s x
    int out_ns, out_rs, out_y0, out_x0, out_s;
    // four stride phases of a transposed convolution in one workgroup (NPH = 4), wavefront f on
    // phase f: its row / column padding and output origin (p / px above are their maxima, which
    // place the shared window; wh_extra = the spread of the row paddings)
    int ph_py[4], ph_px[4], ph_y0[4], ph_x0[4];
    int wh_extra;
    ConeClip clip;   // forward convolutions of cone rows (clip.rows null: none)
    float rWo, rQ;   // 1 / Wo and 1 / (window entries per input row staged): see qdiv
};

// i / d for 0 <= i < 2^21 through r = 1 / d (correctly rounded): (i + 0.5) / d lies at least
// 0.5 / d from an integer, and the product's error, about 2^-22 of the quotient, stays far below
// that; an integer division by a runtime divisor would cost ~30 instructions per use.
__device__ __forceinline__ int qdiv(int i, float r) { return (int)(((float)i + 0.5f) * r); }

template <int BN> struct WinB { static constexpr int BNP = BN + 16; };   // filter row stride: 16 mod 32 banks

template <int K, int S, int BM, int BN, int VEC, int NPH, int NSPLIT>
__global__ __launch_bounds__(256) void k_conv_win(ConvWinArgs a) {
    constexpr int KK = K * K;
    // NPH == 1: the four wavefronts split the tile's positions and channels (NSPLIT 1: channels
    // only, each wavefront taking every position of the tile; NSPLIT 2: two channel halves and the
    // taps, wavefronts f and f + 2 taking every position of half f for the even and the odd taps,
    // their partial tiles then summed in LDS); NPH == 4: wavefront f computes the whole tile of
    // stride phase f
    constexpr bool TSPLIT = NSPLIT == 2;
    constexpr int WAVES_N = NSPLIT == 1 ? 4 : TSPLIT ? 2 : NPH == 1 ? BN / 32 : 1;
    constexpr int WAVES_M = NSPLIT ? 1 : NPH == 1 ? 4 / WAVES_N : 1;
    constexpr int FN = NSPLIT == 1 ? BN / 64 : TSPLIT ? BN / 32 : NPH == 1 ? 2 : BN / 16, FM = BM / (16 * WAVES_M);
    static_assert(NSPLIT != 1 || (NPH == 1 && FN >= 1 && FN * 64 == BN), "channel split");
    static_assert(!TSPLIT || (NPH == 1 && FN * 32 == BN), "tap split");
    static_assert(FM >= 1 && FM * 16 * WAVES_M == BM, "tile");
    static_assert(NPH == 1 || (NPH == 4 && S == 1), "phases");
    constexpr int NLD = VEC == 4 ? NLD4 : NLD1;
    constexpr int BNP = WinB<BN>::BNP;
    constexpr int BQ = BN / 4;                       // float4 per filter row of the tile
    constexpr int WROWS = NPH * KK * CG;             // filter rows (phase, tap, channel) per stage
    constexpr int NW = (WROWS * BQ + 255) / 256;     // float4 filter loads per thread and stage
    // native vectors: copies of HIP's float4 struct out of an array keep the array in scratch
    typedef typename std::conditional<VEC == 4, floatx4, float>::type vec_t;

    extern __shared__ float sm[];
    float* s_w = sm;                    // [NPH][KK][CG][BNP]
    float* s_x = sm + WROWS * BNP;      // [CG][PL]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // wavefront's position and channel block (NPH == 4: the whole tile, for phase `wave`)
    const int wm = NPH == 1 ? wave % WAVES_M : 0, wn = TSPLIT ? (wave & 1) : NPH == 1 ? wave / WAVES_M : 0;
    constexpr int WNC = FN * 16;   // channels per wavefront
    const int r = blockIdx.x / a.mtiles, mt = blockIdx.x - r * a.mtiles;
    const int n0 = blockIdx.y * BN;
    const int P = a.Ho * a.Wo, m0 = mt * BM;
    const int y_first = m0 / a.Wo;
    const int y_last = (min(m0 + BM, P) - 1) / a.Wo;
    const int WH = S * (y_last - y_first) + K + a.wh_extra;
    const int iy0 = S * y_first - a.p;                   // input row of window row 0
    const int wy_lo = max(0, -iy0), wy_hi = min(WH, a.Hi - iy0);
    const int nvr = max(0, wy_hi - wy_lo);
    const long HiWi = (long)a.Hi * a.Wi;

    // this thread's share of a stage's window: offsets in the input row and in LDS (-1: none;
    // such a slot still loads the row's first element, so that no load is conditional)
    const int Q = a.Wi / VEC;
    const int per_c = nvr * Q, total = CG * per_c;
    const float rpc = 1.f / (float)max(per_c, 1);
    int goff[NLD], loff[NLD];
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        const int e = tid + 256 * i;
        goff[i] = 0;
        loff[i] = -1;
        if (e < total) {
            const int c = qdiv(e, rpc), rem = e - c * per_c;
            const int row = qdiv(rem, a.rQ), q = rem - row * Q;
            const int j = q * VEC + a.CO;
            goff[i] = (int)(c * HiWi) + (iy0 + wy_lo + row) * a.Wi + q * VEC;
            loff[i] = c * a.PL + (wy_lo + row) * a.RS + (VEC == 4 ? j / S : (j % S) * a.WS + j / S);
        }
    }
    const float* Grow = a.G + (long)r * a.ldG;
    const float* Wn = a.Wt + n0;
    // filter slots: row (tap, channel) e / BQ, float4 e % BQ of the tile's BN filters
    constexpr bool W_FULL = WROWS * BQ % 256 == 0;

    vec_t xv[NLD];
    floatx4 wv[NW];
#define MNB_WIN_LOAD(g_)                                                                          \
    {                                                                                             \
        const float* src_ = Grow + (long)(g_) * CG * HiWi;                                        \
        _Pragma("unroll") for (int i = 0; i < NLD; ++i)                                           \
            xv[i] = *reinterpret_cast<const vec_t*>(src_ + goff[i]);                              \
        const float* wsrc_ = Wn + (long)(g_) * WROWS * a.Co;                                      \
        _Pragma("unroll") for (int i = 0; i < NW; ++i) {                                          \
            const int e_ = W_FULL ? tid + 256 * i : min(tid + 256 * i, WROWS * BQ - 1);           \
            wv[i] = *reinterpret_cast<const floatx4*>(wsrc_ + (e_ / BQ) * a.Co + (e_ % BQ) * 4);   \
        }                                                                                         \
    }
#define MNB_WIN_STORE()                                                                           \
    {                                                                                             \
        _Pragma("unroll") for (int i = 0; i < NLD; ++i) {                                         \
            if (loff[i] >= 0) {                                                                   \
                if constexpr (VEC == 4) {                                                         \
                    if constexpr (S == 1) {                                                       \
                        *reinterpret_cast<floatx4*>(s_x + loff[i]) = xv[i];                        \
                    } else { /* columns j, j+2 to phase 0, j+1, j+3 to phase 1 */                 \
                        *reinterpret_cast<floatx2*>(s_x + loff[i]) = floatx2{xv[i].x, xv[i].z};          \
                        *reinterpret_cast<floatx2*>(s_x + loff[i] + a.WS) = floatx2{xv[i].y, xv[i].w};   \
                    }                                                                             \
                } else {                                                                          \
                    s_x[loff[i]] = xv[i];                                                         \
                }                                                                                 \
            }                                                                                     \
        }                                                                                         \
        _Pragma("unroll") for (int i = 0; i < NW; ++i) {                                          \
            const int e_ = tid + 256 * i;                                                         \
            if (W_FULL || e_ < WROWS * BQ)                                                        \
                *reinterpret_cast<floatx4*>(s_w + (e_ / BQ) * BNP + (e_ % BQ) * 4) = wv[i];        \
        }                                                                                         \
    }

    // lane bases of this wavefront's position fragments (lanes 16c..16c+15: channel c of a quad)
    int xb[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int m = m0 + wm * FM * 16 + i * 16 + (lane & 15);
        xb[i] = (lane >> 4) * a.PL;
        if (m < P) {
            const int y = qdiv(m, a.rWo), x = m - y * a.Wo;
            xb[i] += S * (y - y_first) * a.RS + x;
        }
    }
    const int wb = (lane >> 4) * BNP + wn * WNC + (lane & 15);
    // this wavefront's phase: extra window rows above its first one, column offset, output origin
    int row_off = 0, c0p = a.CO - a.px, out_y0 = a.out_y0, out_x0 = a.out_x0;
    if constexpr (NPH == 4) {
        const int f = __builtin_amdgcn_readfirstlane(wave);
        const int py = f == 0 ? a.ph_py[0] : f == 1 ? a.ph_py[1] : f == 2 ? a.ph_py[2] : a.ph_py[3];
        const int px = f == 0 ? a.ph_px[0] : f == 1 ? a.ph_px[1] : f == 2 ? a.ph_px[2] : a.ph_px[3];
        out_y0 = f == 0 ? a.ph_y0[0] : f == 1 ? a.ph_y0[1] : f == 2 ? a.ph_y0[2] : a.ph_y0[3];
        out_x0 = f == 0 ? a.ph_x0[0] : f == 1 ? a.ph_x0[1] : f == 2 ? a.ph_x0[2] : a.ph_x0[3];
        row_off = a.p - py;
        c0p = a.CO - px;
    }
    const float* s_wf = s_w + (NPH == 4 ? wave : 0) * KK * CG * BNP;

    floatx4 acc[FN][FM];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int i = 0; i < FM; ++i) acc[j][i] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int ng = a.n_groups;
    MNB_WIN_LOAD(0)
    for (int i = tid; i < CG * a.PL; i += 256) s_x[i] = 0.f;
    __syncthreads();
    MNB_WIN_STORE()
    __syncthreads();
    for (int g = 0; g < ng; ++g) {
        if (g + 1 < ng) MNB_WIN_LOAD(g + 1)
        // taps as a loop (not unrolled): unrolled, the compiler keeps every tap's LDS addresses in
        // registers across the stages, which halves the wavefronts a SIMD can hold
        const int t_first = TSPLIT ? __builtin_amdgcn_readfirstlane(wave >> 1) : 0;
#pragma unroll 1
        for (int t = t_first; t < KK; t += TSPLIT ? 2 : 1) {
            const int ky = t / K, kx = t - ky * K;
            const int tc = kx + c0p;
            const int toff = (ky + row_off) * a.RS + (tc % S) * a.WS + tc / S;
            const float* wt = s_wf + t * CG * BNP + wb;
            const float* xt = s_x + toff;
#pragma unroll
            for (int cq = 0; cq < CG / 4; ++cq) {
                float wf[FN], pf[FM];
#pragma unroll
                for (int j = 0; j < FN; ++j) wf[j] = wt[cq * 4 * BNP + j * 16];
#pragma unroll
                for (int i = 0; i < FM; ++i) pf[i] = xt[xb[i] + cq * 4 * a.PL];
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
                        acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(wf[j], pf[i], acc[j][i], 0, 0, 0);
            }
        }
        if (g + 1 < ng) {
            __syncthreads();   // stage g consumed
            MNB_WIN_STORE()
            __syncthreads();
        }
    }

    if constexpr (TSPLIT) {
        // the odd taps' partial tile added to the even taps' one (wavefront f + 2 to f) through LDS
        // (the stages' space), lane-major so that consecutive lanes write consecutive words;
        // wavefronts 0 and 1 store their channel halves
        constexpr int TILE = FN * FM * 4 * 64;
        __syncthreads();   // the last stage is consumed
        float* red = sm + (wave & 1) * TILE;
        if (wave >= 2) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v) red[((j * FM + i) * 4 + v) * 64 + lane] = acc[j][i][v];
        }
        __syncthreads();
        if (wave >= 2) return;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[j][i][v] += red[((j * FM + i) * 4 + v) * 64 + lane];
    }

    // result lanes: channel n0 + wn WNC + 16 j + 4 (lane / 16) + v, position m0 + ... + lane % 16
#undef MNB_WIN_LOAD
#undef MNB_WIN_STORE
    float bias[FN][4];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            bias[j][v] = a.bias ? a.bias[n0 + wn * WNC + j * 16 + 4 * (lane >> 4) + v] : 0.f;
    float* Cr = a.C + (long)r * a.ldC + (long)(n0 + wn * WNC + 4 * (lane >> 4)) * a.out_ns;
    int moff[FM];
    bool mzero[FM];   // position outside the node of a cone row: written 0
    int coy = 0, cox = 0;
    if (a.clip.rows) cone_origin(a.clip, r, coy, cox);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int m = m0 + wm * FM * 16 + i * 16 + (lane & 15);
        const int y = qdiv(m, a.rWo), x = m - y * a.Wo;
        moff[i] = m < P ? (out_y0 + a.out_s * y) * a.out_rs + out_x0 + a.out_s * x : -1;
        mzero[i] = a.clip.rows && !(coy + y >= 0 && coy + y < a.clip.H && cox + x >= 0 && cox + x < a.clip.W);
    }
    if (a.acc) {
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            if (moff[i] < 0) continue;
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float* q = Cr + (long)(j * 16 + v) * a.out_ns + moff[i];
                    *q += mzero[i] ? 0.f : acc[j][i][v] + bias[j][v];
                }
        }
    } else {
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            if (moff[i] < 0) continue;
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Cr[(long)(j * 16 + v) * a.out_ns + moff[i]] = mzero[i] ? 0.f : acc[j][i][v] + bias[j][v];
        }
    }
}

// Bank score of a plane stride: the largest number of distinct words one LDS bank serves for the
// first position fragment at tap (0, 0), under 64 banks per wavefront and 32 per half.
int bank_score(int PL, int RS, int S, int Wo) {
    int worst64 = 0, worst32 = 0;
    int words[64];
    for (int l = 0; l < 64; ++l) {
        const int m = l & 15, y = m / Wo, x = m - y * Wo;
        words[l] = (l >> 4) * PL + S * y * RS + x;
    }
    for (int nb : {64, 32}) {
        for (int h = 0; h < 64; h += nb) {
            int cnt[64] = {0};
            for (int l = h; l < h + nb; ++l) {
                bool dup = false;
                for (int o = h; o < l; ++o) dup = dup || words[o] == words[l];
                if (!dup) cnt[words[l] % nb]++;
            }
            int w = 0;
            for (int b = 0; b < nb; ++b) w = cnt[b] > w ? cnt[b] : w;
            if (nb == 64) worst64 = w > worst64 ? w : worst64;
            else worst32 = w > worst32 ? w : worst32;
        }
    }
    return worst64 + worst32;
}

// One launch of the window kernel over a virtual convolution: input [M][Cin][Hi][Wi] (row stride
// ldG), K x K taps of stride S, paddings py / px, output grid Ho x Wo of Cout channels placed as
// described in ConvWinArgs, filters Wt [Cin/8][K*K][8][Cout].  false: shape not covered.
struct WinConv {
    const float* G; float* C; const float* Wt; const float* bias;
    int Cin, Hi, Wi, Cout, Ho, Wo, K, S, py, px;
    long ldG, ldC;
    int out_ns, out_rs, out_y0, out_x0, out_s;
    ConeClip clip;
    // nph = 4: the four stride phases at once (filters Wt [Cin/8][4][K*K][8][Cout]); py / px and
    // out_y0 / out_x0 above are then unused
    int nph;
    int ph_py[4], ph_px[4], ph_y0[4], ph_x0[4];
    // only the whole-grid tile (grids of 129 to 144 positions, 64 channels at a time, 3x3 / 1):
    // every position of a row in one workgroup, its wavefronts split along the channels
    bool only_grid;
};

bool launch_win(const WinConv& w, int M, bool accumulate, hipStream_t st, bool check_only) {
    if (w.Wt == nullptr || w.Cin % CG != 0) return false;
    const int BN = w.Cout % 64 == 0 ? 64 : (w.Cout % 32 == 0 ? 32 : 0);
    if (BN == 0) return false;
    const int K = w.K, S = w.S, nph = w.nph == 4 ? 4 : 1;
    const bool ks31 = K == 3 && S == 1, ks42 = K == 4 && S == 2, ks32 = K == 3 && S == 2, ks21 = K == 2 && S == 1;
    if (!(ks31 || ks42 || ks32 || ks21) || w.Ho <= 0 || w.Wo <= 0) return false;
    if (nph == 4 && !ks21) return false;
    const int P = w.Ho * w.Wo;
    // grids of 129 to 144 positions: one workgroup per row holds them all (9 fragments per
    // wavefront, no idle tile), its filters staged once per row
    const bool grid = nph == 1 && BN == 64 && ks31 && P > 128 && P <= 144;
    if (w.only_grid && !grid) return false;
    // stride-2 grids of 81 to 112 positions and 3x3 / 1 grids of at most 48 into 32 channels
    // (ConvBig's 10x10 forward cones, its 6x6 transposed windows): one tile of 16 P / 16 positions
    // per row (96 or 112 for the stride-2 ones), each wavefront pair holding every position of its
    // channel half, the taps split between the pair (a 64- or 128-position tile would leave 22-75%
    // of its lanes idle)
    const bool tsplit = nph == 1 && BN == 32 && ((ks42 && P > 80 && P <= 112) || (ks31 && P <= 48));
    // otherwise positions per workgroup: 128, unless 64 wastes fewer lanes on the last tile (or a
    // wavefront holding a whole tile of 64 channels would need more accumulators)
    const int BM = grid ? 144 : tsplit ? (ks42 ? (P <= 96 ? 96 : 112) : cdiv(P, 16) * 16)
                 : cdiv(P, 64) * 64 < cdiv(P, 128) * 128 || (nph == 4 && BN == 64) ? 64 : 128;
    // phases in one workgroup: the window spans every phase's rows and columns
    int py = w.py, px = w.px, extra = 0;
    if (nph == 4) {
        int lo = w.ph_py[0];
        py = w.ph_py[0];
        px = w.ph_px[0];
        for (int f = 1; f < 4; ++f) {
            py = std::max(py, w.ph_py[f]);
            lo = std::min(lo, w.ph_py[f]);
            px = std::max(px, w.ph_px[f]);
        }
        extra = py - lo;
    }
    const int mtiles = cdiv(P, BM);
    const bool vec = w.Wi % 4 == 0 && w.ldG % 4 == 0 && ((uintptr_t)w.G & 15) == 0;
    // rows of the largest window over the tiles
    int WHmax = 0;
    for (int mt = 0; mt < mtiles; ++mt) {
        const int yf = mt * BM / w.Wo, yl = (std::min((mt + 1) * BM, P) - 1) / w.Wo;
        WHmax = std::max(WHmax, S * (yl - yf) + K + extra);
    }
    ConvWinArgs a{};
    a.G = w.G; a.C = w.C; a.Wt = w.Wt; a.bias = w.bias;
    a.ldG = w.ldG; a.ldC = w.ldC;
    a.Hi = w.Hi; a.Wi = w.Wi; a.Co = w.Cout; a.Ho = w.Ho; a.Wo = w.Wo; a.p = py; a.px = px;
    a.wh_extra = extra;
    for (int f = 0; f < 4; ++f) {
        a.ph_py[f] = w.ph_py[f]; a.ph_px[f] = w.ph_px[f]; a.ph_y0[f] = w.ph_y0[f]; a.ph_x0[f] = w.ph_x0[f];
    }
    a.n_groups = w.Cin / CG;
    a.mtiles = mtiles; a.acc = accumulate;
    a.out_ns = w.out_ns; a.out_rs = w.out_rs; a.out_y0 = w.out_y0; a.out_x0 = w.out_x0; a.out_s = w.out_s;
    a.clip = w.clip;
    a.rWo = 1.f / (float)w.Wo;
    a.CO = px > 0 ? (px + 3) & ~3 : 0;
    int pxlo = px;
    if (nph == 4)
        for (int f = 0; f < 4; ++f) pxlo = std::min(pxlo, w.ph_px[f]);
    const int need = std::max(a.CO + w.Wi, a.CO - pxlo + S * (w.Wo - 1) + K);
    const int JW = cdiv(need, 4 * S) * 4 * S;
    a.RS = JW;
    a.WS = JW / S;
    int best = -1, best_score = 1 << 30;
    for (int t = 0; t < 16; ++t) {
        const int PL = WHmax * a.RS + 4 * t;
        const int sc = bank_score(PL, a.RS, S, w.Wo);
        if (sc < best_score) { best_score = sc; best = PL; }
    }
    a.PL = best;
    const int BNP = BN + 16;
    size_t lds = ((size_t)nph * K * K * CG * BNP + (size_t)CG * a.PL) * sizeof(float);
    if (tsplit) lds = std::max(lds, (size_t)2 * (BN / 32) * (BM / 16) * 4 * 64 * sizeof(float));   // partial tiles
    if (lds > WIN_LDS_MAX) return false;
    // window loads per thread and stage
    const int Q = vec ? w.Wi / 4 : w.Wi;
    a.rQ = 1.f / (float)Q;
    const long loads = (long)CG * std::min(WHmax, w.Hi) * Q;
    if (loads > 256L * (vec ? NLD4 : NLD1)) return false;
    if ((long)M * mtiles > 0x7fffffffL) return false;
    if (check_only || M <= 0) return true;
    const dim3 dgrid((unsigned)(M * mtiles), w.Cout / BN), blk(256);
    if (grid) {
        if (vec) hipLaunchKernelGGL((k_conv_win<3, 1, 144, 64, 4, 1, 1>), dgrid, blk, lds, st, a);
        else hipLaunchKernelGGL((k_conv_win<3, 1, 144, 64, 1, 1, 1>), dgrid, blk, lds, st, a);
        MNB_HIP(hipGetLastError());
        return true;
    }
    if (tsplit) {
#define MNB_WINT(K_, S_, BM_) \
    if (vec) hipLaunchKernelGGL((k_conv_win<K_, S_, BM_, 32, 4, 1, 2>), dgrid, blk, lds, st, a); \
    else hipLaunchKernelGGL((k_conv_win<K_, S_, BM_, 32, 1, 1, 2>), dgrid, blk, lds, st, a)
        if (ks42) { if (BM == 112) { MNB_WINT(4, 2, 112); } else { MNB_WINT(4, 2, 96); } }
        else if (BM == 16) { MNB_WINT(3, 1, 16); }
        else if (BM == 32) { MNB_WINT(3, 1, 32); }
        else { MNB_WINT(3, 1, 48); }
#undef MNB_WINT
        MNB_HIP(hipGetLastError());
        return true;
    }
    if (nph == 4) {
#define MNB_WIN4(BM_, BN_, V_) hipLaunchKernelGGL((k_conv_win<2, 1, BM_, BN_, V_, 4, 0>), dgrid, blk, lds, st, a)
        if (BN == 64) { if (vec) MNB_WIN4(64, 64, 4); else MNB_WIN4(64, 64, 1); }
        else if (BM == 128) { if (vec) MNB_WIN4(128, 32, 4); else MNB_WIN4(128, 32, 1); }
        else { if (vec) MNB_WIN4(64, 32, 4); else MNB_WIN4(64, 32, 1); }
#undef MNB_WIN4
        MNB_HIP(hipGetLastError());
        return true;
    }
#define MNB_WIN(K_, S_, BM_, BN_, V_) \
    hipLaunchKernelGGL((k_conv_win<K_, S_, BM_, BN_, V_, 1, 0>), dgrid, blk, lds, st, a)
#define MNB_WIN_V(K_, S_, BM_, BN_) \
    if (vec) MNB_WIN(K_, S_, BM_, BN_, 4); else MNB_WIN(K_, S_, BM_, BN_, 1)
#define MNB_WIN_T(K_, S_)                                                   \
    if (BM == 128) { if (BN == 64) { MNB_WIN_V(K_, S_, 128, 64); } else { MNB_WIN_V(K_, S_, 128, 32); } } \
    else { if (BN == 64) { MNB_WIN_V(K_, S_, 64, 64); } else { MNB_WIN_V(K_, S_, 64, 32); } }
    if (ks31) { MNB_WIN_T(3, 1); }
    else if (ks42) { MNB_WIN_T(4, 2); }
    else if (ks32) { MNB_WIN_T(3, 2); }
    else { MNB_WIN_T(2, 1); }
#undef MNB_WIN_T
#undef MNB_WIN_V
#undef MNB_WIN
    MNB_HIP(hipGetLastError());
    return true;
}

// Forward convolutions of input planes of at most this many elements stay with the gather GEMM (the
// plane stays in the caches between its re-reads, and the window kernel's filter staging weighs
// more on the few positions of a tile), unless the whole output grid fits one workgroup's tile
// (ConvBig's 10x10 -> 12x12 forward cones).  The transposed convolutions gain from the window
// kernel at every plane size measured (8x8 and up).
constexpr int WIN_MIN_PLANE = 129;

}  // namespace

bool launch_conv_forward_win(const ConvGeom& g, const float* G, float* C, int M, bool accumulate, hipStream_t st,
                             const ConeClip* clip) {
    if ((kernel_variants() & MNB_VAR_NO_WIN_CONV) != 0 || g.p < 0) return false;
    WinConv w{};
    w.only_grid = g.Hi * g.Wi < WIN_MIN_PLANE;
    w.G = G; w.C = C; w.Wt = g.Wt; w.bias = g.b;
    w.Cin = g.Ci; w.Hi = g.Hi; w.Wi = g.Wi; w.Cout = g.Co; w.Ho = g.Ho; w.Wo = g.Wo;
    w.K = g.k; w.S = g.s; w.py = g.p; w.px = g.p;
    w.ldG = (long)g.Ci * g.Hi * g.Wi; w.ldC = (long)g.Co * g.Ho * g.Wo;
    w.out_ns = g.Ho * g.Wo; w.out_rs = g.Wo; w.out_y0 = 0; w.out_x0 = 0; w.out_s = 1;
    w.clip = clip ? *clip : ConeClip{};
    return launch_win(w, M, accumulate, st, false);
}

bool launch_conv_backsub_win(const ConvGeom& g, const float* A, float* C, int M, bool accumulate, hipStream_t st) {
    if ((kernel_variants() & MNB_VAR_NO_WIN_CONV) != 0) return false;
    // the four phases of a stride-2 layer in one launch, where they share taps and grid
    if (g.s == 2 && g.n_phase == 4 && g.Wt4 != nullptr) {
        WinConv w{};
        w.G = A; w.C = C; w.Wt = g.Wt4; w.bias = nullptr;
        w.Cin = g.Co; w.Hi = g.Ho; w.Wi = g.Wo; w.Cout = g.Ci; w.Ho = g.ph[0].nY; w.Wo = g.ph[0].nX;
        w.K = g.ph[0].Ty; w.S = 1;
        w.ldG = (long)g.Co * g.Ho * g.Wo; w.ldC = (long)g.Ci * g.Hi * g.Wi;
        w.out_ns = g.Hi * g.Wi; w.out_rs = g.Wi; w.out_s = g.s;
        w.nph = 4;
        for (int f = 0; f < 4; ++f) {
            const ConvPhase& ph = g.ph[f];
            w.ph_py[f] = ph.Ty - 1 - ph.q0y;
            w.ph_px[f] = ph.Tx - 1 - ph.q0x;
            w.ph_y0[f] = ph.Y0;
            w.ph_x0[f] = ph.X0;
        }
        if (launch_win(w, M, accumulate, st, true)) {
            launch_win(w, M, accumulate, st, false);
            return true;
        }
    }
    // every phase must be covered before any is launched
    WinConv ws[16];
    int n = 0;
    for (int f = 0; f < g.n_phase; ++f) {
        const ConvPhase& ph = g.ph[f];
        if (ph.nY <= 0 || ph.nX <= 0) continue;
        if (ph.Ty != ph.Tx || ph.Ty == 0) return false;   // a phase without taps still writes zeros
        WinConv w{};
        w.G = A; w.C = C; w.Wt = ph.Wt; w.bias = nullptr;
        w.Cin = g.Co; w.Hi = g.Ho; w.Wi = g.Wo; w.Cout = g.Ci; w.Ho = ph.nY; w.Wo = ph.nX;
        w.K = ph.Ty; w.S = 1; w.py = ph.Ty - 1 - ph.q0y; w.px = ph.Tx - 1 - ph.q0x;
        w.ldG = (long)g.Co * g.Ho * g.Wo; w.ldC = (long)g.Ci * g.Hi * g.Wi;
        w.out_ns = g.Hi * g.Wi; w.out_rs = g.Wi; w.out_y0 = ph.Y0; w.out_x0 = ph.X0; w.out_s = g.s;
        if (!launch_win(w, M, accumulate, st, true)) return false;
        ws[n++] = w;
    }
    if (n == 0) return false;
    for (int f = 0; f < n; ++f) launch_win(ws[f], M, accumulate, st, false);
    return true;
}

}  // namespace mnb
