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

// i / d for 0 <= i < 2^16, 0 < d <= 2^10 through a float reciprocal: (i + 0.5) / d lies at least
// 0.5 / d from an integer, far above the rounding of the product.
__device__ __forceinline__ int fdivs(int i, float rd) { return (int)(((float)i + 0.5f) * rd); }

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
    for (int c0 = 0; c0 < Co; c0 += FCO) {
        __syncthreads();   // the previous channels' window is consumed
        if (rb < t.RB && RP > 0) {
            // a fixed window column per thread, RP window rows per pass
            if (srow < RP) {
#pragma unroll 4
                for (int rr = srow; rr < FCO * WY; rr += RP) {
                    const int co = fdivs(rr, rWY), wy = rr - co * WY;   // independent passes: loads batch
                    const int y = y0 + wy;
                    float v = 0.f;
                    if (sxok && c0 + co < Co && y >= 0 && y < Ho) v = Ar[(long)(c0 + co) * HoWo + y * Wo + sx];
                    s_a[rr * WX + scol] = v;
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
        const float* ap = s_a + dy0 * WX + dx0;
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
    if (!act || Y >= Hi) return;
    float* Cr = C + r * (long)CI * Hi * Wi + (long)Y * Wi + X;
#pragma unroll
    for (int c = 0; c < CI; ++c) {
        float* q = Cr + (long)c * Hi * Wi;
        if (X < Wi) q[0] = acc ? q[0] + o0[c] : o0[c];
        if (X + 1 < Wi) q[1] = acc ? q[1] + o1[c] : o1[c];
    }
}

// out[r][co][y][x] (+)= b[co] + sum_{ci, ky, kx} W[co][ci][ky][kx] G[r][ci][y - p + ky][x - p + kx]
// (G positions outside [0, Hi) x [0, Wi) are zero padding).
template <int CI, int K>
__global__ __launch_bounds__(FT) void k_conv_first(const float* __restrict__ G, float* __restrict__ C,
                                                   const float* __restrict__ W, const float* __restrict__ bias, int M,
                                                   int Hi, int Wi, int Co, int Ho, int Wo, int p, int acc,
                                                   FirstTile t, ConeClip clip) {
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
        for (int i = pix; i < CI * win; i += per) {
            const int wr = fdivs(i, rWX), wx = i - wr * WX;
            const int ci = fdivs(wr, rWY), wy = wr - ci * WY;
            const int Y = Y0 + wy, X = X0 + wx;
            float v = 0.f;
            if (r < M && Y >= 0 && Y < Hi && X >= 0 && X < Wi) v = Gr[(long)ci * Hi * Wi + Y * Wi + X];
            s_g[i] = v;
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
        if (x < Wo) o[0] = acc ? o[0] + s0 : s0;
        if (two) o[1] = acc ? o[1] + s1 : s1;
    }
}

bool launch_convT_first(const ConvGeom& g, const float* A, float* C, int M, bool accumulate, hipStream_t st) {
    if (g.s != 1 || g.Ci > 4 || g.k != 3 || (kernel_variants() & MNB_VAR_NO_FIRST_CONV)) return false;
    if (M <= 0) return true;
    const FirstTile t = first_tile(g.Hi, g.Wi);
    const size_t lds = (size_t)t.RB * FCO * (t.TH + 2) * (t.TW + 3) * sizeof(float);
    const long blocks = (long)cdiv(M, t.RB) * t.tiles_x * t.tiles_y;
    MNB_CHECK(blocks < (1L << 31), MNB_EDEVICE, "first-layer transposed convolution: grid too large");
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
    const long blocks = (long)cdiv(M, t.RB) * t.tiles_x * t.tiles_y;
    MNB_CHECK(blocks < (1L << 31), MNB_EDEVICE, "first-layer convolution: grid too large");
#define MNB_CF1(CI_)                                                                                              \
    hipLaunchKernelGGL((k_conv_first<CI_, 3>), dim3((unsigned)blocks), dim3(FT), lds, st, G, C, g.W, g.b, M, g.Hi,   \
                       g.Wi, g.Co, g.Ho, g.Wo, g.p, (int)accumulate, t, clip ? *clip : ConeClip{})
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
