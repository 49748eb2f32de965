// Row-resident implicit-GEMM convolutions on v_mfma_f32_16x16x4_f32 for layers
// whose coefficient rows fit in LDS (ConvSmall's second convolution, the ResNet
// block convolutions).
//
// Back-substitution through a convolution (Eq. 2) and the forward product of
// its adjoint are, per row, small GEMMs over (channels x positions) with the
// layer's weights as one operand.  Each wavefront stages one row into LDS with
// a zero halo, so every tap reads the row from LDS instead of gathering it again
// from global memory; the workgroup's four wavefronts share the weights in LDS
// and walk disjoint rows.  Per row the K-reduction order is fixed, so a row's
// result does not depend on the other rows of the batch.
//   transposed (k_convT_rows): per stride phase, D[ci][pos] = sum over (tap, co)
//       of W_phase[tap][co][ci] * A_row[co][yb - ty][xb - tx]
//   forward    (k_conv_rows):  D[co][pos] = sum over (ky, kx, ci) of
//       Wf[co][(ky, kx, ci)] * G_row[ci][s y - p + ky][s x - p + kx] + b[co]
#include "kernels.h"
#include "../../include/mnbab.h"

#include <stdlib.h>

#include <algorithm>
#include <type_traits>

namespace mnb {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int RT = 256;                 // threads: 4 wavefronts, one row each at a time
constexpr size_t ROW_LDS_MAX = 128 * 1024;

// Wavefront-scope ordering of the row buffer between staging and use.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exact n / d for 0 <= n < 2^22 via a float reciprocal and one correction each way.
struct Div {
    int d;
    float inv;
    __device__ explicit Div(int d_) : d(d_), inv(1.0f / (float)d_) {}
    __device__ __forceinline__ int operator()(int n) const {
        int q = (int)((float)n * inv);
        if ((q + 1) * d <= n) ++q;
        if (q * d > n) --q;
        return q;
    }
};

// One row of up to 256 PF floats (length a multiple of 4) held as PF float4 per lane, so
// that the next row's global loads are in flight while the current row is computed.
template <int PF>
struct RowFetch {
    f4 v[PF];
    __device__ __forceinline__ void fetch(const float* base, long r, int rowlen, bool ok, int lane) {
        const f4* s4 = reinterpret_cast<const f4*>(base + (ok ? r : 0) * rowlen);
        const int n4 = rowlen >> 2;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int i = lane + 64 * u;
            v[u] = (ok && i < n4) ? s4[i] : f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    // element e = c*HW + y*W + x  ->  lds[c*CS + (y + hy)*Wq + x + hx]
    __device__ __forceinline__ void stash(float* lds, int rowlen, int lane, const Div& dHW, const Div& dW, int HW,
                                          int W, int CS, int Wq, int hy, int hx) const {
        const int n4 = rowlen >> 2;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int i = lane + 64 * u;
            if (i < n4) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = 4 * i + q, c = dHW(e), rem = e - c * HW, y = dW(rem), x = rem - y * W;
                    lds[c * CS + (y + hy) * Wq + x + hx] = v[u][q];
                }
            }
        }
    }
    __device__ __forceinline__ void stash_dense(float* lds, int rowlen, int lane) const {
        const int n4 = rowlen >> 2;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int i = lane + 64 * u;
            if (i < n4) *reinterpret_cast<f4*>(lds + 4 * i) = v[u];
        }
    }
};

struct RowPh {
    int Y0, X0, nY, nX, Ty, Tx, q0y, q0x, woff;
};

struct ConvTRowsArgs {
    const float* A; float* C; long M; int acc;
    int Ci, Hi, Wi, Co, Ho, Wo, s;
    int hy, hx, Hp, Wq, CS, RP; // padded row Co x CS (CS >= Hp Wq), halo hy, hx before the first position
    int n_phase; RowPh ph[4]; const float* Wsrc[4];
    int wtot;
};

template <int NT, int C4, int PF>   // C4 = Co / 4; rows of at most 256 PF floats
__global__ __launch_bounds__(RT) void k_convT_rows(ConvTRowsArgs a) {
    extern __shared__ float sm[];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
    float* s_W = sm;
    float* s_row = sm + a.wtot + wave * a.RP;
    for (int f = 0; f < a.n_phase; ++f) {
        const int n = a.ph[f].Ty * a.ph[f].Tx * a.Co * a.Ci;
        for (int i = t; i < n; i += RT) s_W[a.ph[f].woff + i] = a.Wsrc[f][i];
    }
    for (int i = lane; i < a.RP; i += 64) s_row[i] = 0.f;
    __syncthreads();
    const int HoWo = a.Ho * a.Wo, HpWq = a.CS, HiWi = a.Hi * a.Wi;
    const int rowA = a.Co * HoWo;
    const long ldC = (long)a.Ci * HiWi;
    const Div dHoWo(HoWo), dWo(a.Wo);
    const long stride = (long)gridDim.x * 4;
    long r = (long)blockIdx.x * 4 + wave;
    RowFetch<PF> pf;
    pf.fetch(a.A, r, rowA, r < a.M, lane);
    for (; r < a.M; r += stride) {
        pf.stash(s_row, rowA, lane, dHoWo, dWo, HoWo, a.Wo, HpWq, a.Wq, a.hy, a.hx);
        wave_lds_sync();
        pf.fetch(a.A, r + stride, rowA, r + stride < a.M, lane);
        float* dst = a.C + r * ldC;
        for (int f = 0; f < a.n_phase; ++f) {
            const RowPh P = a.ph[f];
            const int npos = P.nY * P.nX;
            if (npos <= 0) continue;
            if (P.Ty * P.Tx <= 0) {
                // positions no tap reaches (kernel smaller than the stride): zero coefficient
                if (!a.acc)
                    for (int idx = lane; idx < a.Ci * npos; idx += 64) {
                        const int ci = idx / npos, n = idx - ci * npos, i = n / P.nX, jx = n - i * P.nX;
                        dst[(long)ci * HiWi + (P.Y0 + a.s * i) * a.Wi + P.X0 + a.s * jx] = 0.f;
                    }
                continue;
            }
            const int ntile = (npos + 15) >> 4;
            for (int ct = 0; ct < a.Ci; ct += 16) {
                // one group of NA position tiles (NA = NT, or the phase's remainder)
                auto group = [&](int n0, auto na_c) {
                    constexpr int NA = decltype(na_c)::value;
                    int pb[NA];
#pragma unroll
                    for (int j = 0; j < NA; ++j) {
                        int n = (n0 + j) * 16 + lr;
                        n = n < npos ? n : npos - 1;
                        const int i = n / P.nX, jx = n - i * P.nX;
                        pb[j] = (P.q0y + i + a.hy) * a.Wq + P.q0x + jx + a.hx;
                    }
                    f4 acc[NA];
#pragma unroll
                    for (int j = 0; j < NA; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
                    // per tap, the C4 groups of 4 output channels are unrolled so that all of
                    // the tap's LDS reads are in flight before its MFMAs
                    const float* wl = s_W + P.woff + ct + lr + lk * a.Ci;
                    const float* rl = s_row + lk * HpWq;
                    for (int ty = 0; ty < P.Ty; ++ty)
                        for (int tx = 0; tx < P.Tx; ++tx) {
                            const int tap = ty * P.Tx + tx;
                            const float* wt = wl + (long)tap * a.Co * a.Ci;
                            const float* rt = rl - ty * a.Wq - tx;
                            float av[C4], bv[C4][NA];
#pragma unroll
                            for (int c = 0; c < C4; ++c) {
                                av[c] = wt[4 * c * a.Ci];
#pragma unroll
                                for (int j = 0; j < NA; ++j) bv[c][j] = rt[4 * c * HpWq + pb[j]];
                            }
#pragma unroll
                            for (int c = 0; c < C4; ++c)
#pragma unroll
                                for (int j = 0; j < NA; ++j)
                                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c], bv[c][j], acc[j], 0, 0, 0);
                        }
                    // D: lane holds ci = ct + 4 lk + v at position (n0 + j) * 16 + lr
#pragma unroll
                    for (int j = 0; j < NA; ++j) {
                        const int n = (n0 + j) * 16 + lr;
                        if (n < npos) {
                            const int i = n / P.nX, jx = n - i * P.nX;
                            float* q = dst + (long)(ct + 4 * lk) * HiWi + (P.Y0 + a.s * i) * a.Wi + P.X0 + a.s * jx;
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                float* qq = q + (long)v * HiWi;
                                *qq = a.acc ? *qq + acc[j][v] : acc[j][v];
                            }
                        }
                    }
                };
                int n0 = 0;
                for (; n0 + NT <= ntile; n0 += NT) group(n0, std::integral_constant<int, NT>{});
                const int rem = ntile - n0;
                if (NT > 3 && rem == 3) group(n0, std::integral_constant<int, (NT > 3 ? 3 : 1)>{});
                if (NT > 2 && rem == 2) group(n0, std::integral_constant<int, (NT > 2 ? 2 : 1)>{});
                if (rem == 1) group(n0, std::integral_constant<int, 1>{});
            }
        }
        wave_lds_sync();   // every lane is done with this row before the next one is staged
    }
}

struct ConvRowsArgs {
    const float* G; float* C; const float* bias; const float* Wf; long M; int acc;
    int Ci, Hi, Wi, Co, Ho, Wo, k, s, p;
    int Hp, Wq, RP, K, KW;      // padded row Ci x Hp x Wq; K = k k Ci; KW = LDS weight row stride
};

template <int NT, int MT, int C4, int PF>   // C4 = Ci / 4; rows of at most 256 PF floats
__global__ __launch_bounds__(RT) void k_conv_rows(ConvRowsArgs a) {
    extern __shared__ float sm[];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
    float* s_W = sm;                              // [Co][KW]
    float* s_b = sm + (long)a.Co * a.KW;          // [Co] bias
    float* s_row = s_b + ((a.Co + 3) & ~3) + wave * a.RP;
    for (int i = t; i < a.Co * a.K; i += RT) {
        const int co = i / a.K;
        s_W[co * a.KW + (i - co * a.K)] = a.Wf[i];
    }
    for (int i = t; i < a.Co; i += RT) s_b[i] = a.bias[i];
    for (int i = lane; i < a.RP; i += 64) s_row[i] = 0.f;
    __syncthreads();
    const int HoWo = a.Ho * a.Wo, HpWq = a.Hp * a.Wq, HiWi = a.Hi * a.Wi;
    const int rowG = a.Ci * HiWi;
    const long ldC = (long)a.Co * HoWo;
    const int ntile = (HoWo + 15) >> 4;
    const Div dHiWi(HiWi), dWi(a.Wi);
    const bool dense = a.p == 0 && a.Hp == a.Hi && a.Wq == a.Wi;   // padded layout == row layout
    const long stride = (long)gridDim.x * 4;
    long r = (long)blockIdx.x * 4 + wave;
    RowFetch<PF> pf;
    pf.fetch(a.G, r, rowG, r < a.M, lane);
    for (; r < a.M; r += stride) {
        if (dense)
            pf.stash_dense(s_row, rowG, lane);
        else
            pf.stash(s_row, rowG, lane, dHiWi, dWi, HiWi, a.Wi, HpWq, a.Wq, a.p, a.p);
        wave_lds_sync();
        pf.fetch(a.G, r + stride, rowG, r + stride < a.M, lane);
        float* dst = a.C + r * ldC;
        for (int ct = 0; ct < a.Co; ct += 16 * MT) {
            for (int n0 = 0; n0 < ntile; n0 += NT) {
                int pb[NT];
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    int n = (n0 + j) * 16 + lr;
                    n = n < HoWo ? n : HoWo - 1;
                    const int y = n / a.Wo, x = n - y * a.Wo;
                    pb[j] = a.s * y * a.Wq + a.s * x;
                }
                f4 acc[MT][NT];
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int j = 0; j < NT; ++j) acc[m][j] = f4{0.f, 0.f, 0.f, 0.f};
                const float* wrow[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    int co = ct + m * 16 + lr;
                    co = co < a.Co ? co : a.Co - 1;
                    wrow[m] = s_W + (long)co * a.KW + lk;   // + 4 ks (K ordered (ky, kx, ci))
                }
                // per tap, the C4 groups of 4 input channels are unrolled so that all of the
                // tap's LDS reads are in flight before its MFMAs
                const float* rl = s_row + lk * HpWq;
                for (int ky = 0; ky < a.k; ++ky)
                    for (int kx = 0; kx < a.k; ++kx) {
                        const int kb = (ky * a.k + kx) * a.Ci;
                        // the tap's row offset opaque to the compiler (one register, not one
                        // induction register per read)
                        int tb = ky * a.Wq + kx;
                        asm volatile("" : "+v"(tb));
                        float av[C4][MT], bv[C4][NT];
#pragma unroll
                        for (int c = 0; c < C4; ++c) {
#pragma unroll
                            for (int m = 0; m < MT; ++m) av[c][m] = wrow[m][kb + 4 * c];
#pragma unroll
                            for (int j = 0; j < NT; ++j) bv[c][j] = rl[tb + pb[j] + 4 * c * HpWq];
                        }
#pragma unroll
                        for (int c = 0; c < C4; ++c)
#pragma unroll
                            for (int m = 0; m < MT; ++m)
#pragma unroll
                                for (int j = 0; j < NT; ++j)
                                    acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c][m], bv[c][j], acc[m][j], 0, 0, 0);
                    }
                // D: lane holds co = ct + 16 m + 4 lk + v at position (n0 + j) * 16 + lr.  The next
                // row's loads have arrived by now: wait for them before the stores, so that
                // nothing is outstanding when the next row is staged
                vmem_drain();
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int co = ct + m * 16 + 4 * lk + v;
                        if (co >= a.Co) continue;
                        const float b = s_b[co];
#pragma unroll
                        for (int j = 0; j < NT; ++j) {
                            const int n = (n0 + j) * 16 + lr;
                            if (n < HoWo) {
                                float* q = dst + (long)co * HoWo + n;
                                const float val = acc[m][j][v] + b;
                                *q = a.acc ? *q + val : val;
                            }
                        }
                    }
            }
        }
        wave_lds_sync();
    }
}

// Transposed convolution of rows whose input grid is small (at most 32 positions, up to
// 16 taps, stride 2): per output channel ci a GEMM T[pos][tap] = sum_co A[co][pos] W[co][ci][tap]
// over the row's own positions (no halo or stride-phase padding), then a col2im gather of the
// at most 4 taps reaching each output.  Each wavefront owns a row at a time; the row is the
// MFMA A operand straight from registers (loaded one row ahead), the weights are the B
// operand from LDS, and T goes through a double-buffered per-wavefront LDS tile.
struct ConvTTapArgs {
    const float* A; float* C; const float* W; long M; int acc;
    int Ci, Hi, Wi, Co, Ho, Wo, k, s, p;
};

constexpr int TT = 512;   // threads: 8 wavefronts
constexpr int TLD = 17;   // T row stride (positions x 16 taps, padded)

template <int MT, int K4, int NQ>   // MT: 16-position tiles, K4 = Co / 4, NQ: outputs per lane per channel
__global__ __launch_bounds__(TT) void k_convT_tap(ConvTTapArgs a) {
    constexpr int NTO = 4;                    // taps reaching an output (kernel <= 2 x stride 2)
    constexpr int TB = (16 * MT + 1) * TLD;   // one T tile: 16 MT position rows and a zero row
    constexpr int TZ = 16 * MT * TLD;         // the zero row (never written): target of absent taps
    extern __shared__ float sm[];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
    const int kk = a.k * a.k, HoWo = a.Ho * a.Wo, HiWi = a.Hi * a.Wi;
    float* s_W = sm;                                         // [Ci][Co][16] B operand, taps padded
    float* s_T = sm + a.Ci * a.Co * 16 + wave * 2 * TB;      // [2][16 MT + 1][TLD]
    if (lane == 0) s_T[TZ] = s_T[TB + TZ] = 0.f;
    for (int i = t; i < a.Ci * a.Co * 16; i += TT) {
        const int tap = i & 15, cc = i >> 4, co = cc % a.Co, ci = cc / a.Co;
        s_W[i] = tap < kk ? a.W[((long)co * a.Ci + ci) * kk + tap] : 0.f;
    }
    // per owned output q = lane + 64 i of a channel: its taps' T entries (TZ, a zero: none)
    int tix[NQ][NTO];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int q = lane + 64 * i;
        const bool qv = q < HiWi;
        const int Y = qv ? q / a.Wi : 0, X = qv ? q - Y * a.Wi : 0;
        const int Yp = Y + a.p, Xp = X + a.p;
#pragma unroll
        for (int u = 0; u < NTO; ++u) {
            const int ky = Yp % a.s + (u >> 1) * a.s, kx = Xp % a.s + (u & 1) * a.s;
            const int y = (Yp - ky) / a.s, x = (Xp - kx) / a.s;
            const bool tv = qv && ky < a.k && kx < a.k && Yp >= ky && Xp >= kx && y < a.Ho && x < a.Wo;
            tix[i][u] = tv ? (y * a.Wo + x) * TLD + ky * a.k + kx : TZ;
        }
    }
    const long stride = (long)gridDim.x * (TT / 64);
    long r = (long)blockIdx.x * (TT / 64) + wave;
    // A operand of the row: lane (lr, lk) holds A[co = 4 ks + lk][pos = 16 mt + lr]
    float nx[MT][K4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ks = 0; ks < K4; ++ks) {
            const int pos = 16 * mt + lr;
            nx[mt][ks] = (r < a.M && pos < HoWo) ? a.A[r * a.Co * HoWo + (4 * ks + lk) * HoWo + pos] : 0.f;
        }
    __syncthreads();
    const long ldC = (long)a.Ci * HiWi;
    for (; r < a.M; r += stride) {
        float av[MT][K4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int ks = 0; ks < K4; ++ks) av[mt][ks] = nx[mt][ks];
        if (r + stride < a.M) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int ks = 0; ks < K4; ++ks) {
                    const int pos = 16 * mt + lr;
                    nx[mt][ks] = pos < HoWo ? a.A[(r + stride) * a.Co * HoWo + (4 * ks + lk) * HoWo + pos] : 0.f;
                }
        }
        float* dst = a.C + r * ldC;
        auto channel = [&](int ci) {
            float* T = s_T + (ci & 1) * TB;
            f4 acc[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
            const float* wb = s_W + (long)ci * a.Co * 16 + lk * 16 + lr;
#pragma unroll
            for (int ks = 0; ks < K4; ++ks) {
                const float b = wb[ks * 64];   // W[co = 4 ks + lk][ci][tap = lr]
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt][ks], b, acc[mt], 0, 0, 0);
            }
            // lane holds T[pos = 16 mt + 4 lk + v][tap = lr]
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) T[(16 * mt + 4 * lk + v) * TLD + lr] = acc[mt][v];
            wave_lds_sync();
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                const int q = lane + 64 * i;
                if (q < HiWi) {
                    float sum = 0.f;
#pragma unroll
                    for (int u = 0; u < NTO; ++u) sum += T[tix[i][u]];
                    float* o = dst + (long)ci * HiWi + q;
                    *o = a.acc ? *o + sum : sum;
                }
            }
        };
        // the loads of the next row have arrived by the middle of this one: wait for them
        // there, so that nothing is outstanding at the top of the next row
        const int half = a.Ci / 2;
        for (int ci = 0; ci < half; ++ci) channel(ci);
        vmem_drain();
        for (int ci = half; ci < a.Ci; ++ci) channel(ci);
    }
}

// Forward convolution with two wavefronts per row (32 output channels): each wavefront of a
// pair stages half of the row into the pair's LDS buffer and computes 16 of the output
// channels, so a workgroup of eight wavefronts holds four rows and the CU twice as many
// wavefronts as with one row per wavefront.  Per row the K-reduction order is that of
// k_conv_rows (taps, then channel groups).
__device__ __forceinline__ void block_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int PT = 512;   // threads: 4 pairs of wavefronts

template <int NT, int C4, int PF>   // C4 = Ci / 4; PF: float4 per lane for half a row
__global__ __launch_bounds__(PT, 4) void k_conv_pair(ConvRowsArgs a) {
    constexpr int NP = PT / 128;
    extern __shared__ float sm[];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, pair = wave >> 1, half = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    float* s_W = sm;                              // [Co][KW]
    float* s_b = sm + (long)a.Co * a.KW;          // [Co] bias
    float* s_row = s_b + ((a.Co + 3) & ~3) + pair * a.RP;
    for (int i = t; i < a.Co * a.K; i += PT) {
        const int co = i / a.K;
        s_W[co * a.KW + (i - co * a.K)] = a.Wf[i];
    }
    for (int i = t; i < a.Co; i += PT) s_b[i] = a.bias[i];
    for (int i = lane + 64 * half; i < a.RP; i += 128) s_row[i] = 0.f;
    const int HoWo = a.Ho * a.Wo, HpWq = a.Hp * a.Wq, HiWi = a.Hi * a.Wi;
    const int rowG = a.Ci * HiWi;
    const long ldC = (long)a.Co * HoWo;
    const int ntile = (HoWo + 15) >> 4;
    const bool dense = a.p == 0 && a.Hp == a.Hi && a.Wq == a.Wi;   // padded layout == row layout
    const int n4 = rowG >> 2, n4h = (n4 + 1) >> 1;
    const int q0 = half * n4h, q1 = min(n4, q0 + n4h);              // this wavefront's float4 range
    const long stride = (long)gridDim.x * NP;
    const long rb = (long)blockIdx.x * NP;
    // iterations of the workgroup (every wavefront takes part in every barrier)
    const long niter = a.M > rb ? (a.M - rb + stride - 1) / stride : 0;
    const long r0 = rb + pair;
    f4 v[PF];
    auto fetch = [&](long r) {
        const f4* s4 = reinterpret_cast<const f4*>(a.G + (r < a.M ? r : 0) * rowG);
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int i = q0 + lane + 64 * u;
            v[u] = (r < a.M && i < q1) ? s4[i] : f4{0.f, 0.f, 0.f, 0.f};
        }
    };
    fetch(r0);
    __syncthreads();
    for (long it = 0; it < niter; ++it) {
        const long r = r0 + it * stride;
        // stage this wavefront's half of the row
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int i = q0 + lane + 64 * u;
            if (i < q1) {
                if (dense) {
                    *reinterpret_cast<f4*>(s_row + 4 * i) = v[u];
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int e = 4 * i + q, c = e / HiWi, rem = e - c * HiWi, y = rem / a.Wi, x = rem - y * a.Wi;
                        s_row[c * HpWq + (y + a.p) * a.Wq + x + a.p] = v[u][q];
                    }
                }
            }
        }
        block_lds_sync();   // the pair's row is complete
        fetch(r + stride);
        if (r < a.M) {
            float* dst = a.C + r * ldC;
            const int co_w = 16 * half + lr;   // A operand row: output channel
            const float* wrow = s_W + (long)co_w * a.KW + lk;   // + 4 ks (K ordered (ky, kx, ci))
            const float* rl = s_row + lk * HpWq;
            for (int n0 = 0; n0 < ntile; n0 += NT) {
                int pb[NT];
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    int n = (n0 + j) * 16 + lr;
                    n = n < HoWo ? n : HoWo - 1;
                    const int y = n / a.Wo, x = n - y * a.Wo;
                    pb[j] = a.s * y * a.Wq + a.s * x;
                }
                f4 acc[NT];
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
                for (int ky = 0; ky < a.k; ++ky)
                    for (int kx = 0; kx < a.k; ++kx) {
                        const int kb = (ky * a.k + kx) * a.Ci;
                        // the tap's row offset, opaque to the compiler: every read address is
                        // then this plus a uniform channel offset, instead of one induction
                        // register per (channel group, tile), and the tap's reads all fit in
                        // registers at once
                        int tb = ky * a.Wq + kx;
                        asm volatile("" : "+v"(tb));
                        float av[C4], bv[C4][NT];
#pragma unroll
                        for (int c = 0; c < C4; ++c) {
                            av[c] = wrow[kb + 4 * c];
#pragma unroll
                            for (int j = 0; j < NT; ++j) bv[c][j] = rl[tb + pb[j] + 4 * c * HpWq];
                        }
#pragma unroll
                        for (int c = 0; c < C4; ++c)
#pragma unroll
                            for (int j = 0; j < NT; ++j)
                                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c], bv[c][j], acc[j], 0, 0, 0);
                    }
                // D: lane holds co = 16 half + 4 lk + v at position (n0 + j) * 16 + lr; the next
                // row's loads have arrived by now: wait for them before the stores
                vmem_drain();
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    const int co = 16 * half + 4 * lk + vv;
                    const float b = s_b[co];
#pragma unroll
                    for (int j = 0; j < NT; ++j) {
                        const int n = (n0 + j) * 16 + lr;
                        if (n < HoWo) {
                            float* q = dst + (long)co * HoWo + n;
                            const float val = acc[j][vv] + b;
                            *q = a.acc ? *q + val : val;
                        }
                    }
                }
            }
        } else {
            vmem_drain();
        }
        block_lds_sync();   // both wavefronts are done with the row before the next is staged
    }
}

int row_grid(long M) {
    const long nb = (M + 3) / 4;
    return (int)(nb < 2048 ? nb : 2048);
}

}  // namespace

// Tap-GEMM form of the transposed convolution for small input grids; false when the shape
// does not fit it.
static bool launch_convT_tap(const ConvGeom& g, const float* A, float* C, int M, bool accumulate, hipStream_t st) {
    const bool off = (kernel_variants() & (MNB_VAR_NO_TAP_CONVT | MNB_VAR_NO_ROW_CONV)) != 0;
    const int HoWo = g.Ho * g.Wo, HiWi = g.Hi * g.Wi;
    if (off || g.s != 2 || g.k > 4 || g.Co != 32 || HoWo > 32 || HiWi > 192 || g.Ci < 2) return false;
    ConvTTapArgs a{};
    a.A = A; a.C = C; a.W = g.W; a.M = M; a.acc = accumulate;
    a.Ci = g.Ci; a.Hi = g.Hi; a.Wi = g.Wi; a.Co = g.Co; a.Ho = g.Ho; a.Wo = g.Wo; a.k = g.k; a.s = g.s; a.p = g.p;
    const int mt = (HoWo + 15) / 16, nq = (HiWi + 63) / 64;
    const size_t lds = ((size_t)g.Ci * g.Co * 16 + (size_t)(TT / 64) * 2 * (16 * mt + 1) * TLD) * sizeof(float);
    if (lds > ROW_LDS_MAX) return false;
    if (M <= 0) return true;
    const long nb = (M + TT / 64 - 1) / (TT / 64);
    const dim3 grid((int)(nb < 512 ? nb : 512));
#define MNB_TT(MT_, NQ_) hipLaunchKernelGGL((k_convT_tap<MT_, 8, NQ_>), grid, dim3(TT), lds, st, a)
    if (mt == 1) {
        if (nq == 1) MNB_TT(1, 1); else if (nq == 2) MNB_TT(1, 2); else MNB_TT(1, 3);
    } else {
        if (nq == 1) MNB_TT(2, 1); else if (nq == 2) MNB_TT(2, 2); else MNB_TT(2, 3);
    }
#undef MNB_TT
    MNB_HIP(hipGetLastError());
    return true;
}

bool launch_conv_backsub_rows(const ConvGeom& g, const float* A, float* C, int M, bool accumulate,
                              hipStream_t st) {
    if (launch_convT_tap(g, A, C, M, accumulate, st)) return true;
    const bool off = (kernel_variants() & MNB_VAR_NO_ROW_CONV) != 0;
    if (off || g.Ci % 16 != 0 || (g.Co != 16 && g.Co != 32 && g.Co != 64) || g.n_phase > 4) return false;
    const int rowA = g.Co * g.Ho * g.Wo;
    if (rowA % 4 != 0 || rowA > 4096 || ((uintptr_t)A & 15) != 0) return false;
    ConvTRowsArgs a{};
    a.A = A; a.C = C; a.M = M; a.acc = accumulate;
    a.Ci = g.Ci; a.Hi = g.Hi; a.Wi = g.Wi; a.Co = g.Co; a.Ho = g.Ho; a.Wo = g.Wo; a.s = g.s;
    int hy = 0, hx = 0, ey = g.Ho, ex = g.Wo, woff = 0, maxtile = 0;
    a.n_phase = 0;
    for (int f = 0; f < g.n_phase; ++f) {
        const ConvPhase& ph = g.ph[f];
        if (ph.nY <= 0 || ph.nX <= 0) continue;
        RowPh& q = a.ph[a.n_phase];
        q.Y0 = ph.Y0; q.X0 = ph.X0; q.nY = ph.nY; q.nX = ph.nX; q.Ty = ph.Ty; q.Tx = ph.Tx;
        q.q0y = ph.q0y; q.q0x = ph.q0x; q.woff = woff;
        a.Wsrc[a.n_phase] = ph.Wp;
        a.n_phase++;
        if (ph.Ty <= 0 || ph.Tx <= 0) continue;
        woff += ph.Ty * ph.Tx * g.Co * g.Ci;
        hy = std::max(hy, ph.Ty - 1 - ph.q0y);
        hx = std::max(hx, ph.Tx - 1 - ph.q0x);
        ey = std::max(ey, ph.q0y + ph.nY);
        ex = std::max(ex, ph.q0x + ph.nX);
        maxtile = std::max(maxtile, (ph.nY * ph.nX + 15) / 16);
    }
    if (a.n_phase == 0) return false;
    a.hy = hy; a.hx = hx; a.Hp = hy + ey; a.Wq = hx + ex;
    // channel stride = 16 mod 32 words: the four k-groups of a wavefront's read fall on
    // different LDS banks
    a.CS = a.Hp * a.Wq + ((16 - (a.Hp * a.Wq) % 32) + 32) % 32;
    a.RP = (g.Co * a.CS + 3) & ~3;
    a.wtot = (woff + 3) & ~3;
    const size_t lds = ((size_t)a.wtot + 4 * (size_t)a.RP) * sizeof(float);
    if (lds > ROW_LDS_MAX) return false;
    if (M <= 0) return true;
    const dim3 grid(row_grid(M));
    const int c4 = g.Co / 4;
    const bool pf4 = g.Co * g.Ho * g.Wo <= 1024;
    const int nt = maxtile >= 4 ? 4 : maxtile >= 2 ? 2 : 1;
#define MNB_CT(NT_, C4_)                                                                  \
    if (pf4) hipLaunchKernelGGL((k_convT_rows<NT_, C4_, 4>), grid, dim3(RT), lds, st, a);  \
    else hipLaunchKernelGGL((k_convT_rows<NT_, C4_, 16>), grid, dim3(RT), lds, st, a)
#define MNB_CT_NT(C4_)          \
    if (nt == 4) MNB_CT(4, C4_); \
    else if (nt == 2) MNB_CT(2, C4_); \
    else MNB_CT(1, C4_)
    if (c4 == 4) { MNB_CT_NT(4); }
    else if (c4 == 8) { MNB_CT_NT(8); }
    else { MNB_CT_NT(16); }
#undef MNB_CT_NT
#undef MNB_CT
    MNB_HIP(hipGetLastError());
    return true;
}

bool launch_conv_forward_rows(const ConvGeom& g, const float* G, float* C, int M, bool accumulate,
                              hipStream_t st) {
    const bool off = (kernel_variants() & MNB_VAR_NO_ROW_CONV) != 0;
    if (off || g.Co % 16 != 0 || (g.Ci != 16 && g.Ci != 32 && g.Ci != 64)) return false;
    const int rowG = g.Ci * g.Hi * g.Wi;
    if (rowG % 4 != 0 || rowG > 4096 || ((uintptr_t)G & 15) != 0) return false;
    ConvRowsArgs a{};
    a.G = G; a.C = C; a.bias = g.b; a.Wf = g.Wf; a.M = M; a.acc = accumulate;
    a.Ci = g.Ci; a.Hi = g.Hi; a.Wi = g.Wi; a.Co = g.Co; a.Ho = g.Ho; a.Wo = g.Wo;
    a.k = g.k; a.s = g.s; a.p = g.p;
    a.Hp = std::max(g.Hi + 2 * g.p, (g.Ho - 1) * g.s + g.k);
    a.Wq = std::max(g.Wi + 2 * g.p, (g.Wo - 1) * g.s + g.k);
    a.RP = (g.Ci * a.Hp * a.Wq + 3) & ~3;
    a.K = g.k * g.k * g.Ci;
    a.KW = a.K + 4;
    const size_t lds = ((size_t)g.Co * a.KW + ((g.Co + 3) & ~3) + 4 * (size_t)a.RP) * sizeof(float);
    if (lds > ROW_LDS_MAX) return false;
    if (M <= 0) return true;
    const bool no_pair = (kernel_variants() & MNB_VAR_NO_PAIR_CONV) != 0;
    if (!no_pair && g.Co == 32 && (rowG / 4 + 1) / 2 <= 64 * 8) {
        // two wavefronts per row; half a row is at most 8 float4 per lane
        const long nb = (M + 3) / 4;
        const dim3 grid2((int)(nb < 512 ? nb : 512));
        const int ntile = (g.Ho * g.Wo + 15) / 16;
        const int nt = ntile >= 2 ? 2 : 1;
        const int c4 = g.Ci / 4;
        const int pfn = ((rowG / 4 + 1) / 2 + 63) / 64;   // float4 per lane for half a row
#define MNB_CP_PF(NT_, C4_)                                                                        \
    if (pfn <= 4) hipLaunchKernelGGL((k_conv_pair<NT_, C4_, 4>), grid2, dim3(PT), lds, st, a);      \
    else if (pfn <= 6) hipLaunchKernelGGL((k_conv_pair<NT_, C4_, 6>), grid2, dim3(PT), lds, st, a); \
    else hipLaunchKernelGGL((k_conv_pair<NT_, C4_, 8>), grid2, dim3(PT), lds, st, a)
        if (c4 == 4) { if (nt == 2) { MNB_CP_PF(2, 4); } else { MNB_CP_PF(1, 4); } }
        else if (c4 == 8) { if (nt == 2) { MNB_CP_PF(2, 8); } else { MNB_CP_PF(1, 8); } }
        else { if (nt == 2) { MNB_CP_PF(2, 16); } else { MNB_CP_PF(1, 16); } }
#undef MNB_CP_PF
        MNB_HIP(hipGetLastError());
        return true;
    }
    const dim3 grid(row_grid(M));
    const int ntile = (g.Ho * g.Wo + 15) / 16;
    const int nt = ntile >= 4 ? 4 : ntile >= 2 ? 2 : 1;
    const int mt = g.Co % 32 == 0 ? 2 : 1;
    const int c4 = g.Ci / 4;
    const bool pf4 = g.Ci * g.Hi * g.Wi <= 1024;
#define MNB_CF(NT_, MT_, C4_)                                                                  \
    if (pf4) hipLaunchKernelGGL((k_conv_rows<NT_, MT_, C4_, 4>), grid, dim3(RT), lds, st, a);   \
    else hipLaunchKernelGGL((k_conv_rows<NT_, MT_, C4_, 16>), grid, dim3(RT), lds, st, a)
#define MNB_CF_NT(MT_, C4_)             \
    if (nt == 4) MNB_CF(4, MT_, C4_);    \
    else if (nt == 2) MNB_CF(2, MT_, C4_); \
    else MNB_CF(1, MT_, C4_)
#define MNB_CF_MT(C4_)                  \
    if (mt == 2) { MNB_CF_NT(2, C4_); }  \
    else { MNB_CF_NT(1, C4_); }
    if (c4 == 4) { MNB_CF_MT(4) }
    else if (c4 == 8) { MNB_CF_MT(8) }
    else { MNB_CF_MT(16) }
#undef MNB_CF_MT
#undef MNB_CF_NT
#undef MNB_CF
    MNB_HIP(hipGetLastError());
    return true;
}

}  // namespace mnb
