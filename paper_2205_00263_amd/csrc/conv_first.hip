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

// Output tile of one row: TW x TH positions with TH TW <= FT; RB rows per workgroup.
struct FirstTile {
    int TW, TH, RB, tiles_x, tiles_y;
};
static FirstTile first_tile(int H, int W) {
    FirstTile t;
    t.TW = W < 32 ? W : 32;
    t.TH = std::min(H, FT / t.TW);
    t.RB = std::max(1, FT / (t.TW * t.TH));
    t.tiles_x = cdiv(W, t.TW);
    t.tiles_y = cdiv(H, t.TH);
    return t;
}

// out[r][ci][Y][X] (+)= sum_{co, ky, kx} A[r][co][Y + p - ky][X + p - kx] W[co][ci][ky][kx]
// (A positions outside [0, Ho) x [0, Wo) are absent).
template <int CI, int K>
__global__ __launch_bounds__(FT) void k_convT_first(const float* __restrict__ A, float* __restrict__ C,
                                                    const float* __restrict__ W, int M, int Hi, int Wi, int Co,
                                                    int Ho, int Wo, int p, int acc, FirstTile t) {
    extern __shared__ float sm[];
    const int WY = t.TH + K - 1, WX = t.TW + K - 1, win = WY * WX;
    const int rb = threadIdx.x / (t.TW * t.TH), pix = threadIdx.x - rb * (t.TW * t.TH);
    const int tile = blockIdx.x % (t.tiles_x * t.tiles_y);
    const long r = (long)(blockIdx.x / (t.tiles_x * t.tiles_y)) * t.RB + rb;
    const int ty0 = (tile / t.tiles_x) * t.TH, tx0 = (tile % t.tiles_x) * t.TW;
    const int Y = ty0 + pix / t.TW, X = tx0 + pix % t.TW;
    const bool act = rb < t.RB && r < M && pix < t.TW * t.TH;
    // window origin on the layer output: y = Y + p - ky for ky = K-1 .. 0
    const int y0 = ty0 + p - (K - 1), x0 = tx0 + p - (K - 1);
    float* s_a = sm + (rb < t.RB ? rb : 0) * FCO * win;
    const float* Ar = A + (act ? r : 0) * (long)Co * Ho * Wo;
    const int HoWo = Ho * Wo;
    float out[CI];
#pragma unroll
    for (int c = 0; c < CI; ++c) out[c] = 0.f;
    for (int c0 = 0; c0 < Co; c0 += FCO) {
        __syncthreads();   // the previous channels' window is consumed
        if (rb < t.RB) {
            for (int i = pix; i < FCO * win; i += t.TW * t.TH) {
                const int co = i / win, rem = i - co * win, wy = rem / WX, wx = rem - wy * WX;
                const int y = y0 + wy, x = x0 + wx;
                float v = 0.f;
                if (r < M && c0 + co < Co && y >= 0 && y < Ho && x >= 0 && x < Wo)
                    v = Ar[(long)(c0 + co) * HoWo + y * Wo + x];
                s_a[i] = v;
            }
        }
        __syncthreads();
        const int nco = Co - c0 < FCO ? Co - c0 : FCO;
        const float* ap = s_a + (Y - ty0) * WX + (X - tx0);
        for (int co = 0; co < nco; ++co) {
            const float* wrow = W + (long)(c0 + co) * CI * K * K;
#pragma unroll
            for (int ky = 0; ky < K; ++ky)
#pragma unroll
                for (int kx = 0; kx < K; ++kx) {
                    // A[y][x] with y = Y + p - ky sits at window row (K - 1 - ky) + (Y - ty0)
                    const float av = ap[co * win + (K - 1 - ky) * WX + (K - 1 - kx)];
#pragma unroll
                    for (int c = 0; c < CI; ++c) out[c] += av * wrow[(c * K + ky) * K + kx];
                }
        }
    }
    if (!act || Y >= Hi || X >= Wi) return;
    float* Cr = C + r * (long)CI * Hi * Wi + (long)Y * Wi + X;
#pragma unroll
    for (int c = 0; c < CI; ++c) {
        float* q = Cr + (long)c * Hi * Wi;
        *q = acc ? *q + out[c] : out[c];
    }
}

// out[r][co][y][x] (+)= b[co] + sum_{ci, ky, kx} W[co][ci][ky][kx] G[r][ci][y - p + ky][x - p + kx]
// (G positions outside [0, Hi) x [0, Wi) are zero padding).
template <int CI, int K>
__global__ __launch_bounds__(FT) void k_conv_first(const float* __restrict__ G, float* __restrict__ C,
                                                   const float* __restrict__ W, const float* __restrict__ bias, int M,
                                                   int Hi, int Wi, int Co, int Ho, int Wo, int p, int acc,
                                                   FirstTile t) {
    extern __shared__ float sm[];
    const int WY = t.TH + K - 1, WX = t.TW + K - 1, win = WY * WX;
    const int rb = threadIdx.x / (t.TW * t.TH), pix = threadIdx.x - rb * (t.TW * t.TH);
    const int tile = blockIdx.x % (t.tiles_x * t.tiles_y);
    const long r = (long)(blockIdx.x / (t.tiles_x * t.tiles_y)) * t.RB + rb;
    const int ty0 = (tile / t.tiles_x) * t.TH, tx0 = (tile % t.tiles_x) * t.TW;
    const int y = ty0 + pix / t.TW, x = tx0 + pix % t.TW;
    const bool act = rb < t.RB && r < M && pix < t.TW * t.TH;
    const int Y0 = ty0 - p, X0 = tx0 - p;   // input window origin
    float* s_g = sm + (rb < t.RB ? rb : 0) * CI * win;
    const float* Gr = G + (r < M ? r : 0) * (long)CI * Hi * Wi;
    if (rb < t.RB) {
        for (int i = pix; i < CI * win; i += t.TW * t.TH) {
            const int ci = i / win, rem = i - ci * win, wy = rem / WX, wx = rem - wy * WX;
            const int Y = Y0 + wy, X = X0 + wx;
            float v = 0.f;
            if (r < M && Y >= 0 && Y < Hi && X >= 0 && X < Wi) v = Gr[(long)ci * Hi * Wi + Y * Wi + X];
            s_g[i] = v;
        }
    }
    __syncthreads();
    if (!act || y >= Ho || x >= Wo) return;
    float in[CI * K * K];
    const float* gp = s_g + (y - ty0) * WX + (x - tx0);
#pragma unroll
    for (int ci = 0; ci < CI; ++ci)
#pragma unroll
        for (int ky = 0; ky < K; ++ky)
#pragma unroll
            for (int kx = 0; kx < K; ++kx) in[(ci * K + ky) * K + kx] = gp[ci * win + ky * WX + kx];
    float* Cr = C + r * (long)Co * Ho * Wo + (long)y * Wo + x;
    for (int co = 0; co < Co; ++co) {
        const float* w = W + (long)co * CI * K * K;
        float s = bias[co];
#pragma unroll
        for (int q = 0; q < CI * K * K; ++q) s += w[q] * in[q];
        float* o = Cr + (long)co * Ho * Wo;
        *o = acc ? *o + s : s;
    }
}

bool launch_convT_first(const ConvGeom& g, const float* A, float* C, int M, bool accumulate, hipStream_t st) {
    if (g.s != 1 || g.Ci > 4 || g.k != 3 || (kernel_variants() & MNB_VAR_NO_FIRST_CONV)) return false;
    if (M <= 0) return true;
    const FirstTile t = first_tile(g.Hi, g.Wi);
    const size_t lds = (size_t)t.RB * FCO * (t.TH + 2) * (t.TW + 2) * sizeof(float);
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

bool launch_conv_first(const ConvGeom& g, const float* G, float* C, int M, bool accumulate, hipStream_t st) {
    if (g.s != 1 || g.Ci > 4 || g.k != 3 || (kernel_variants() & MNB_VAR_NO_FIRST_CONV)) return false;
    if (M <= 0) return true;
    const FirstTile t = first_tile(g.Ho, g.Wo);
    const size_t lds = (size_t)t.RB * g.Ci * (t.TH + 2) * (t.TW + 2) * sizeof(float);
    const long blocks = (long)cdiv(M, t.RB) * t.tiles_x * t.tiles_y;
    MNB_CHECK(blocks < (1L << 31), MNB_EDEVICE, "first-layer convolution: grid too large");
#define MNB_CF1(CI_)                                                                                              \
    hipLaunchKernelGGL((k_conv_first<CI_, 3>), dim3((unsigned)blocks), dim3(FT), lds, st, G, C, g.W, g.b, M, g.Hi,   \
                       g.Wi, g.Co, g.Ho, g.Wo, g.p, (int)accumulate, t)
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
