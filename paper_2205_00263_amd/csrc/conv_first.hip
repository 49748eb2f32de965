// Convolutions with very few input channels (the first layer of CIFAR networks, Ci <= 4), stride 1.
//
// Back-substitution through such a layer (Eq. 2) is a transposed convolution into Ci channels,
// and the adjoint's forward pass a convolution out of them: per output element only Ci k k
// multiply-adds per output channel, so an MFMA tile over Ci would be mostly padding.  These
// kernels use the VALU: one thread per output position, the filter read with wave-uniform
// addresses (scalar loads, SGPR operands of the FMAs), the input tile of several output channels
// (transposed) or of all input channels (forward) staged in LDS, and one coalesced store per
// output plane.  Small outputs (receptive-field windows and cones) put several rows into one
// workgroup.
#include "kernels.h"
#include "../../include/mnbab.h"

#include <algorithm>

namespace mnb {

constexpr int FT = 256;     // threads per workgroup
constexpr int FCO = 8;      // transposed: layer output channels staged per step
constexpr int SB = 8;       // staging loads in flight per thread
typedef float f2 __attribute__((ext_vector_type(2)));

// Output tile of one row: TW x TH positions, each thread two horizontally adjacent ones
// (TW even, TW / 2 * TH <= FT); RB rows per workgroup.
struct FirstTile {
    int TW, TH, RB, tiles_x, tiles_y;
};
static FirstTile first_tile(int H, int W) {
    FirstTile t;
    t.TW = std::min(32, (W + 1) & ~1);
    t.TH = std::min(H, 2 * FT / t.TW);
    t.RB = std::max(1, FT / (t.TW / 2 * t.TH));
    t.tiles_x = cdiv(W, t.TW);
    t.tiles_y = cdiv(H, t.TH);
    return t;
}

// i / d for 0 <= i < 2^16, d > 0 through a float reciprocal: (i + 0.5) / d lies at least 0.5 / d
// from an integer, while the rounding of the reciprocal and of the product moves it by at most
// about 2^-23 (i + 0.5) / d, below that for every i < 2^22.
__device__ __forceinline__ int fdivs(int i, float rd) { return (int)(((float)i + 0.5f) * rd); }

// The transposed convolution's products for one thread's output pair over nco staged channels:
// ap points at the pair's window (rows dy0.., columns dx0..) of the first staged channel, channel
// planes win floats apart.  Channels, then ky, then kx: every tile shape sums in this order.
template <int CI, int K>
__device__ __forceinline__ void convT_first_taps(const float* ap, int win, int WX, const float* __restrict__ W,
                                                 int c0, int nco, float (&o0)[CI], float (&o1)[CI]) {
#pragma unroll 2
    for (int co = 0; co < nco; ++co) {
        const float* wrow = W + (long)(c0 + co) * CI * K * K;
#pragma unroll
        for (int ky = 0; ky < K; ++ky) {
            // A[y][x] with y = Y + p - ky sits at window row (K - 1 - ky) + dy0; the pair's
            // columns for taps kx are (K - 1 - kx) + dx0 + {0, 1}
            float a[K + 1];
#pragma unroll
            for (int q = 0; q <= K; ++q) a[q] = ap[co * win + (K - 1 - ky) * WX + q];
#pragma unroll
            for (int kx = 0; kx < K; ++kx)
#pragma unroll
                for (int c = 0; c < CI; ++c) {
                    const float w = wrow[(c * K + ky) * K + kx];
                    o0[c] += a[K - 1 - kx] * w;
                    o1[c] += a[K - kx] * w;
                }
        }
    }
}

// Store (or add to) one thread's output pair at (Y, X), X + 1 of row r.
template <int CI>
__device__ __forceinline__ void convT_first_store(float* __restrict__ C, long r, int Hi, int Wi, int Y, int X,
                                                  int acc, float (&o0)[CI], float (&o1)[CI]) {
    float* Cr = C + r * (long)CI * Hi * Wi + (long)Y * Wi + X;
    if (acc) {
        // all previous values in flight together (a position past the plane reads its row's last)
        const int e0 = X < Wi ? 0 : Wi - 1 - X, e1 = X + 1 < Wi ? 1 : Wi - 1 - X;
        float p0[CI], p1[CI];
#pragma unroll
        for (int c = 0; c < CI; ++c) {
            p0[c] = Cr[(long)c * Hi * Wi + e0];
            p1[c] = Cr[(long)c * Hi * Wi + e1];
        }
#pragma unroll
        for (int c = 0; c < CI; ++c) {
            o0[c] += p0[c];
            o1[c] += p1[c];
        }
    }
#pragma unroll
    for (int c = 0; c < CI; ++c) {
        float* q = Cr + (long)c * Hi * Wi;
        if (X < Wi) q[0] = o0[c];
        if (X + 1 < Wi) q[1] = o1[c];
    }
}

// out[r][ci][Y][X] (+)= sum_{co, ky, kx} A[r][co][Y + p - ky][X + p - kx] W[co][ci][ky][kx]
// (A positions outside [0, Ho) x [0, Wo) are absent).
template <int CI, int K>
__global__ __launch_bounds__(FT) void k_convT_first(const float* __restrict__ A, float* __restrict__ C,
                                                    const float* __restrict__ W, int M, int Hi, int Wi, int Co,
                                                    int Ho, int Wo, int p, int acc, FirstTile t) {
    extern __shared__ float sm[];
    const int WY = t.TH + K - 1, WX = t.TW + K, win = WY * WX;   // one spare column: the pair's 4th read
    const int per = t.TW / 2 * t.TH;
    const int rb = threadIdx.x / per, pix = threadIdx.x - rb * per;
    const int tile = blockIdx.x % (t.tiles_x * t.tiles_y);
    const long r = (long)(blockIdx.x / (t.tiles_x * t.tiles_y)) * t.RB + rb;
    const int ty0 = (tile / t.tiles_x) * t.TH, tx0 = (tile % t.tiles_x) * t.TW;
    const int dy0 = pix / (t.TW / 2), dx0 = 2 * (pix % (t.TW / 2));
    const int Y = ty0 + dy0, X = tx0 + dx0;
    const bool act = rb < t.RB && r < M;
    // window origin on the layer output: y = Y + p - ky for ky = K-1 .. 0
    const int y0 = ty0 + p - (K - 1), x0 = tx0 + p - (K - 1);
    float* s_a = sm + (rb < t.RB ? rb : 0) * FCO * win;
    const float* Ar = A + (act ? r : 0) * (long)Co * Ho * Wo;
    const int HoWo = Ho * Wo;
    const float rWX = 1.f / (float)WX, rWY = 1.f / (float)WY;
    // staging map: thread pix owns window column scol of rows srow, srow + RP, ...
    const int RP = per / WX;
    const int srow = fdivs(pix, rWX), scol = pix - srow * WX;
    const int sx = x0 + scol;
    const bool sxok = r < M && sx >= 0 && sx < Wo;
    float o0[CI], o1[CI];
#pragma unroll
    for (int c = 0; c < CI; ++c) o0[c] = o1[c] = 0.f;
    const int nrr = FCO * WY;
    for (int c0 = 0; c0 < Co; c0 += FCO) {
        __syncthreads();   // the previous channels' window is consumed
        if (rb < t.RB && RP > 0) {
            // a fixed window column per thread, RP window rows per pass; SB passes' loads in flight
            // together (every lane loads, from element 0 of its row where the position is absent,
            // and selects afterwards: a load under a branch would wait before the next one)
            if (srow < RP) {
                for (int rr0 = srow; rr0 < nrr; rr0 += SB * RP) {
                    float v[SB];
#pragma unroll
                    for (int u = 0; u < SB; ++u) {
                        const int rr = rr0 + u * RP;
                        const int co = fdivs(rr, rWY), wy = rr - co * WY;
                        const int y = y0 + wy;
                        const bool ok = sxok && rr < nrr && c0 + co < Co && y >= 0 && y < Ho;
                        const float x = Ar[ok ? (long)(c0 + co) * HoWo + y * Wo + sx : 0];
                        v[u] = ok ? x : 0.f;
                    }
#pragma unroll
                    for (int u = 0; u < SB; ++u)
                        if (rr0 + u * RP < nrr) s_a[(rr0 + u * RP) * WX + scol] = v[u];
                }
            }
        } else if (rb < t.RB) {
            for (int i = pix; i < FCO * win; i += per) {
                const int wr = fdivs(i, rWX), wx = i - wr * WX;
                const int co = fdivs(wr, rWY), wy = wr - co * WY;
                const int y = y0 + wy, x = x0 + wx;
                float v = 0.f;
                if (r < M && c0 + co < Co && y >= 0 && y < Ho && x >= 0 && x < Wo)
                    v = Ar[(long)(c0 + co) * HoWo + y * Wo + x];
                s_a[i] = v;
            }
        }
        __syncthreads();
        const int nco = Co - c0 < FCO ? Co - c0 : FCO;
        convT_first_taps<CI, K>(s_a + dy0 * WX + dx0, win, WX, W, c0, nco, o0, o1);
    }
    if (!act || Y >= Hi) return;
    convT_first_store<CI>(C, r, Hi, Wi, Y, X, acc, o0, o1);
}

// Zero source for the direct staging below: window positions outside the layer output (and rows
// past the batch) load from here.
__device__ float g_first_zero[64] = {};

// The same transposed convolution with the window staged by direct global-to-LDS loads: no
// registers hold the data in flight, so a stage's loads all issue at once; FC channels per stage,
// double-buffered, the next stage's loads in flight while this stage's products run.  The block's
// RB windows of FC channel planes lie in LDS as in the kernel above; thread t stages elements t,
// t + FT, ... of that range, so a wavefront's lanes write consecutive words (the direct load's
// layout).  An element's source offset within the stage's channels is the same for every stage
// and is computed once (NPE <= NPX passes, Co a multiple of FC: both checked by the launch);
// window positions outside the layer output, rows past the batch and the slots past the windows
// read the zero source.  TWC > 0: the tile is TWC x THC (strides known to the compiler, whose
// LDS reads then take them as immediate offsets).  Sums in the order above.
template <int CI, int K, int FC, int NPX, int TWC, int THC>
__global__ __launch_bounds__(FT) void k_convT_first_dma(const float* __restrict__ A, float* __restrict__ C,
                                                        const float* __restrict__ W, int M, int Hi, int Wi, int Co,
                                                        int Ho, int Wo, int p, int acc, FirstTile t, int NPE) {
    extern __shared__ float sm[];
    if constexpr (TWC > 0) {
        t.TW = TWC;
        t.TH = THC;
    }
    const int WY = t.TH + K - 1, WX = t.TW + K, win = WY * WX;
    const int per = t.TW / 2 * t.TH;
    const int rb = threadIdx.x / per, pix = threadIdx.x - rb * per;
    const int tile = blockIdx.x % (t.tiles_x * t.tiles_y);
    const long rf = (long)(blockIdx.x / (t.tiles_x * t.tiles_y)) * t.RB;   // the block's first row (< M)
    const long r = rf + rb;
    const int ty0 = (tile / t.tiles_x) * t.TH, tx0 = (tile % t.tiles_x) * t.TW;
    const int dy0 = pix / (t.TW / 2), dx0 = 2 * (pix % (t.TW / 2));
    const int Y = ty0 + dy0, X = tx0 + dx0;
    const bool live = rb < t.RB;
    const bool act = live && r < M;
    const int y0 = ty0 + p - (K - 1), x0 = tx0 + p - (K - 1);
    const int HoWo = Ho * Wo, CHW = Co * HoWo;
    const float* Ab = A + rf * (long)CHW;
    const float rwin = 1.f / (float)win, rWX = 1.f / (float)WX;
    const float* zero = g_first_zero + (threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63);
    int poff[NPX];   // element threadIdx.x + u FT: offset from the stage's first channel plane, or -1
#pragma unroll
    for (int u = 0; u < NPX; ++u) {
        poff[u] = -1;
        if (u >= NPE) continue;   // uniform
        const int e = threadIdx.x + u * FT;
        const int pl = fdivs(e, rwin), w = e - pl * win;   // plane rb' FC + co, position in it
        const int wy = fdivs(w, rWX), wx = w - wy * WX;
        const int eb = pl / FC, co = pl - eb * FC;
        const int y = y0 + wy, x = x0 + wx;
        poff[u] = eb < t.RB && rf + eb < M && y >= 0 && y < Ho && x >= 0 && x < Wo
                      ? eb * CHW + co * HoWo + y * Wo + x
                      : -1;
    }
    const int bstride = NPE * FT;   // floats per buffer
    auto stage = [&](int c0, float* buf) {
        const float* base = Ab + (long)c0 * HoWo;
#pragma unroll
        for (int u = 0; u < NPX; ++u)
            if (u < NPE)
                __builtin_amdgcn_global_load_lds(poff[u] >= 0 ? base + poff[u] : zero, buf + wave + u * FT, 4, 0, 0);
    };
    float o0[CI], o1[CI];
#pragma unroll
    for (int c = 0; c < CI; ++c) o0[c] = o1[c] = 0.f;
    const float* ap = sm + (live ? rb : 0) * FC * win + dy0 * WX + dx0;
    stage(0, sm);
    int cur = 0;
    for (int c0 = 0; c0 < Co; c0 += FC) {
        vmem_drain();      // this thread's loads of the stage have reached LDS
        __syncthreads();   // everyone's; and the other buffer's products are done
        if (c0 + FC < Co) stage(c0 + FC, sm + (cur ^ 1) * bstride);
        if (live) convT_first_taps<CI, K>(ap + cur * bstride, win, WX, W, c0, FC, o0, o1);
        cur ^= 1;
    }
    if (!act || Y >= Hi) return;
    convT_first_store<CI>(C, r, Hi, Wi, Y, X, acc, o0, o1);
}

// out[r][co][y][x] (+)= b[co] + sum_{ci, ky, kx} W[co][ci][ky][kx] G[r][ci][y - p + ky][x - p + kx]
// (G positions outside [0, Hi) x [0, Wi) are zero padding).
template <int CI, int K>
__global__ __launch_bounds__(FT) void k_conv_first(const float* __restrict__ G, float* __restrict__ C,
                                                   const float* __restrict__ W, const float* __restrict__ bias, int M,
                                                   int Hi, int Wi, int Co, int Ho, int Wo, int p, int acc,
                                                   FirstTile t, ConeClip clip, int st2) {
    extern __shared__ float sm[];
    const int WY = t.TH + K - 1, WX = t.TW + K, win = WY * WX;
    const int per = t.TW / 2 * t.TH;
    const int rb = threadIdx.x / per, pix = threadIdx.x - rb * per;
    const int tile = blockIdx.x % (t.tiles_x * t.tiles_y);
    const long r = (long)(blockIdx.x / (t.tiles_x * t.tiles_y)) * t.RB + rb;
    const int ty0 = (tile / t.tiles_x) * t.TH, tx0 = (tile % t.tiles_x) * t.TW;
    const int dy0 = pix / (t.TW / 2), dx0 = 2 * (pix % (t.TW / 2));
    const int y = ty0 + dy0, x = tx0 + dx0;
    const bool act = rb < t.RB && r < M;
    const int Y0 = ty0 - p, X0 = tx0 - p;   // input window origin
    float* s_g = sm + (rb < t.RB ? rb : 0) * CI * win;
    const float* Gr = G + (r < M ? r : 0) * (long)CI * Hi * Wi;
    const float rWX = 1.f / (float)WX, rWY = 1.f / (float)WY;
    if (rb < t.RB) {
        // SB loads in flight together, selected afterwards (as in the transposed kernel)
        const int n = CI * win;
        for (int i0 = pix; i0 < n; i0 += SB * per) {
            float v[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int i = i0 + u * per;
                const int wr = fdivs(i, rWX), wx = i - wr * WX;
                const int ci = fdivs(wr, rWY), wy = wr - ci * WY;
                const int Y = Y0 + wy, X = X0 + wx;
                const bool ok = r < M && i < n && Y >= 0 && Y < Hi && X >= 0 && X < Wi;
                const float x = Gr[ok ? (long)ci * Hi * Wi + Y * Wi + X : 0];
                v[u] = ok ? x : 0.f;
            }
#pragma unroll
            for (int u = 0; u < SB; ++u)
                if (i0 + u * per < n) s_g[i0 + u * per] = v[u];
        }
    }
    __syncthreads();
    if (!act || y >= Ho) return;
    // the pair's inputs: rows dy0 + ky, columns dx0 + 0 .. K
    float in[CI * K * (K + 1)];
    const float* gp = s_g + dy0 * WX + dx0;
#pragma unroll
    for (int ci = 0; ci < CI; ++ci)
#pragma unroll
        for (int ky = 0; ky < K; ++ky)
#pragma unroll
            for (int q = 0; q <= K; ++q) in[(ci * K + ky) * (K + 1) + q] = gp[ci * win + ky * WX + q];
    float* Cr = C + r * (long)Co * Ho * Wo + (long)y * Wo + x;
    const bool two = x + 1 < Wo;
    // cone rows: positions outside the node are written 0
    bool z0 = false, z1 = false;
    if (clip.rows) {
        int oy, ox;
        cone_origin(clip, r, oy, ox);
        const bool yin = oy + y >= 0 && oy + y < clip.H;
        z0 = !(yin && ox + x >= 0 && ox + x < clip.W);
        z1 = !(yin && ox + x + 1 >= 0 && ox + x + 1 < clip.W);
    }
#pragma unroll 2
    for (int co = 0; co < Co; ++co) {
        const float* w = W + (long)co * CI * K * K;
        float s0 = bias[co], s1 = s0;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci)
#pragma unroll
            for (int ky = 0; ky < K; ++ky)
#pragma unroll
                for (int kx = 0; kx < K; ++kx) {
                    const float wv = w[(ci * K + ky) * K + kx];
                    s0 += wv * in[(ci * K + ky) * (K + 1) + kx];
                    s1 += wv * in[(ci * K + ky) * (K + 1) + kx + 1];
                }
        float* o = Cr + (long)co * Ho * Wo;
        if (z0) s0 = 0.f;
        if (z1) s1 = 0.f;
        if (st2) {
            // even plane width, 8-byte aligned output: the pair is one aligned 8-byte word
            if (x < Wo) {
                f2 v = {s0, s1};
                if (acc) {
                    const f2 pv = *reinterpret_cast<const f2*>(o);
                    v = f2{pv.x + s0, pv.y + s1};
                }
                *reinterpret_cast<f2*>(o) = v;
            }
        } else {
            if (x < Wo) o[0] = acc ? o[0] + s0 : s0;
            if (two) o[1] = acc ? o[1] + s1 : s1;
        }
    }
}

bool launch_convT_first(const ConvGeom& g, const float* A, float* C, int M, bool accumulate, hipStream_t st) {
    if (g.s != 1 || g.Ci > 4 || g.k != 3 || (kernel_variants() & MNB_VAR_NO_FIRST_CONV)) return false;
    if (M <= 0) return true;
    const FirstTile t = first_tile(g.Hi, g.Wi);
    const long blocks = (long)cdiv(M, t.RB) * t.tiles_x * t.tiles_y;
    MNB_CHECK(blocks < (1L << 31), MNB_EDEVICE, "first-layer transposed convolution: grid too large");
    {
        // direct staging (the register-staged kernel below serves the remaining shapes)
        constexpr int FCD = 4, NPX = 16;
        const int NPE = cdiv(t.RB * FCD * (t.TH + 2) * (t.TW + 3), FT);
        if (NPE <= NPX && g.Co % FCD == 0 && (long)t.RB * g.Co * g.Ho * g.Wo < (1L << 31)) {
            const size_t lds = (size_t)2 * NPE * FT * sizeof(float);
#define MNB_CTD_(CI_, TW_, TH_)                                                                          \
    hipLaunchKernelGGL((k_convT_first_dma<CI_, 3, FCD, NPX, TW_, TH_>), dim3((unsigned)blocks), dim3(FT), lds, st, A, \
                       C, g.W, M, g.Hi, g.Wi, g.Co, g.Ho, g.Wo, g.p, (int)accumulate, t, NPE)
#define MNB_CTD(CI_)                                                                        \
    if (t.TW == 32 && t.TH == 16) MNB_CTD_(CI_, 32, 16); /* whole 32-wide planes */            \
    else if (t.TW == 16 && t.TH == 16) MNB_CTD_(CI_, 16, 16); /* windows of 16, 10 and 6 */    \
    else if (t.TW == 10 && t.TH == 10) MNB_CTD_(CI_, 10, 10);                                 \
    else if (t.TW == 6 && t.TH == 6) MNB_CTD_(CI_, 6, 6);                                     \
    else MNB_CTD_(CI_, 0, 0)
            switch (g.Ci) {
                case 1: MNB_CTD(1); break;
                case 2: MNB_CTD(2); break;
                case 3: MNB_CTD(3); break;
                default: MNB_CTD(4); break;
            }
#undef MNB_CTD
#undef MNB_CTD_
            MNB_HIP(hipGetLastError());
            return true;
        }
    }
    const size_t lds = (size_t)t.RB * FCO * (t.TH + 2) * (t.TW + 3) * sizeof(float);
#define MNB_CTF(CI_)                                                                                              \
    hipLaunchKernelGGL((k_convT_first<CI_, 3>), dim3((unsigned)blocks), dim3(FT), lds, st, A, C, g.W, M, g.Hi, g.Wi, \
                       g.Co, g.Ho, g.Wo, g.p, (int)accumulate, t)
    switch (g.Ci) {
        case 1: MNB_CTF(1); break;
        case 2: MNB_CTF(2); break;
        case 3: MNB_CTF(3); break;
        default: MNB_CTF(4); break;
    }
#undef MNB_CTF
    MNB_HIP(hipGetLastError());
    return true;
}

bool launch_conv_first(const ConvGeom& g, const float* G, float* C, int M, bool accumulate, hipStream_t st,
                       const ConeClip* clip) {
    if (g.s != 1 || g.Ci > 4 || g.k != 3 || (kernel_variants() & MNB_VAR_NO_FIRST_CONV)) return false;
    if (M <= 0) return true;
    const FirstTile t = first_tile(g.Ho, g.Wo);
    const size_t lds = (size_t)t.RB * g.Ci * (t.TH + 2) * (t.TW + 3) * sizeof(float);
    const int st2 = g.Wo % 2 == 0 && ((uintptr_t)C & 7) == 0;   // pairs as 8-byte stores
    const long blocks = (long)cdiv(M, t.RB) * t.tiles_x * t.tiles_y;
    MNB_CHECK(blocks < (1L << 31), MNB_EDEVICE, "first-layer convolution: grid too large");
#define MNB_CF1(CI_)                                                                                              \
    hipLaunchKernelGGL((k_conv_first<CI_, 3>), dim3((unsigned)blocks), dim3(FT), lds, st, G, C, g.W, g.b, M, g.Hi,   \
                       g.Wi, g.Co, g.Ho, g.Wo, g.p, (int)accumulate, t, clip ? *clip : ConeClip{}, st2)
    switch (g.Ci) {
        case 1: MNB_CF1(1); break;
        case 2: MNB_CF1(2); break;
        case 3: MNB_CF1(3); break;
        default: MNB_CF1(4); break;
    }
#undef MNB_CF1
    MNB_HIP(hipGetLastError());
    return true;
}

}  // namespace mnb
