// FP32 MFMA products of back-substitution (Eq. 2) and of its adjoint.
//
// One generic LDS-staged GEMM  C[m, n] = sum_k A(m, k) B(k, n)  on
// v_mfma_f32_16x16x4_f32, 256 threads (4 wavefronts of 64), with the operand
// element maps supplied by a small "problem" class:
//   FcBack   A = coefficient rows [M, dout], B = W [dout, din]            (a W)
//   FcFwd    A = forward rows [M, din],      B(k, n) = W[n, k]            (g W^T + b)
//   ConvBack A(m, k) gathers the coefficient of the conv output that feeds
//            input position m through tap k (one stride phase per launch:
//            implicit-GEMM transposed convolution), B = phase weights
//   ConvFwd  A(m, k) gathers the input patch (implicit-GEMM convolution)
// The K-reduction order of an output element depends only on (n, K), never
// on M or on neighbouring rows, so a row's result is the same in any batch.
#include "kernels.h"

namespace mnb {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16;

// ------------------------------------------------------------------ problems
struct FcBack {
    static constexpr bool A_MFAST = false;   // A contiguous along k
    static constexpr bool B_NFAST = true;    // B contiguous along n
    const float* A; const float* W; float* C;
    int M, N, K; int acc;
    struct MCtx { long base, cbase; bool ok; };
    __device__ MCtx mctx(int m) const { return {(long)m * K, (long)m * N, m < M}; }
    __device__ float a(const MCtx& c, int k) const { return (c.ok && k < K) ? A[c.base + k] : 0.f; }
    __device__ float b(int k, int n) const { return (k < K && n < N) ? W[(long)k * N + n] : 0.f; }
    static constexpr int tile_ok = 0;
    template <int NA>
    __device__ void a_tile(const MCtx&, int, const int*, float*) const {}
    __device__ void store_ctx(const MCtx& c, int n, float v) const {
        if (c.ok && n < N) {
            float* p = C + c.cbase + n;
            *p = acc ? *p + v : v;
        }
    }
};

struct FcFwd {
    static constexpr bool A_MFAST = false;
    static constexpr bool B_NFAST = false;   // B(k, n) = W[n*K + k], contiguous along k
    const float* A; const float* W; const float* bias; float* C;
    int M, N, K; int acc;
    struct MCtx { long base, cbase; bool ok; };
    __device__ MCtx mctx(int m) const { return {(long)m * K, (long)m * N, m < M}; }
    __device__ float a(const MCtx& c, int k) const { return (c.ok && k < K) ? A[c.base + k] : 0.f; }
    __device__ float b(int k, int n) const { return (k < K && n < N) ? W[(long)n * K + k] : 0.f; }
    static constexpr int tile_ok = 0;
    template <int NA>
    __device__ void a_tile(const MCtx&, int, const int*, float*) const {}
    __device__ void store_ctx(const MCtx& c, int n, float v) const {
        if (c.ok && n < N) {
            float* p = C + c.cbase + n;
            v += bias[n];
            *p = acc ? *p + v : v;
        }
    }
};

struct ConvBack {
    static constexpr bool A_MFAST = true;
    static constexpr bool B_NFAST = true;
    const float* A; float* C;
    const float* Wp; const int2* ktab;
    int M, N, K;          // M = rows*nY*nX, N = Ci, K = Co*Ty*Tx
    int nY, nX, Ho, Wo, ldA, ldC, HiWi, Wi, Y0, X0, s, q0y, q0x;
    int acc;
    struct MCtx { long base; int yb, xb; bool ok; long cbase; };
    __device__ MCtx mctx(int m) const {
        MCtx c;
        c.ok = m < M;
        int mm = c.ok ? m : 0;
        int per = nY * nX;
        int r = mm / per, rem = mm - r * per;
        int i = rem / nX, jx = rem - i * nX;
        c.yb = q0y + i;
        c.xb = q0x + jx;
        c.base = (long)r * ldA + (long)c.yb * Wo + c.xb;
        c.cbase = (long)r * ldC + (long)(Y0 + s * i) * Wi + (X0 + s * jx);
        return c;
    }
    __device__ float a(const MCtx& c, int k) const {
        if (!c.ok || k >= K) return 0.f;
        int2 t = ktab[k];
        int ty = t.y >> 16, tx = t.y & 0xffff;
        int y = c.yb - ty, x = c.xb - tx;
        if ((unsigned)y >= (unsigned)Ho || (unsigned)x >= (unsigned)Wo) return 0.f;
        return A[c.base + t.x];
    }
    __device__ float b(int k, int n) const { return (k < K && n < N) ? Wp[(long)k * N + n] : 0.f; }
    // A elements k0 + ks[i] of one K-tile that lies within a single tap (Co % 16 == 0); K ordered
    // (co / 16, ty, tx, co % 16): the k-tiles of one 16-channel group are its taps in a row
    int tile_ok, Co, Tx, Ty, HoWo;
    template <int NA>
    __device__ void a_tile(const MCtx& c, int k0, const int* ks, float* out) const {
        const int kt = k0 >> 4;
        const int cg = kt / (Ty * Tx), tap = kt - cg * Ty * Tx;
        const int ty = tap / Tx, tx = tap - ty * Tx;
        const int co0 = cg * 16 + (k0 & 15);   // k0 carries the thread's first k within the tile
        const int y = c.yb - ty, x = c.xb - tx;
        const bool ok = c.ok && k0 < K && (unsigned)y < (unsigned)Ho && (unsigned)x < (unsigned)Wo;
        const float* src = A + (c.base + (long)co0 * HoWo - ty * Wo - tx);
#pragma unroll
        for (int i = 0; i < NA; ++i) out[i] = ok ? src[(long)ks[i] * HoWo] : 0.f;
    }
    __device__ void store_ctx(const MCtx& c, int n, float v) const {
        if (c.ok && n < N) {
            float* p = C + c.cbase + (long)n * HiWi;
            *p = acc ? *p + v : v;
        }
    }
};

struct ConvFwd {
    static constexpr bool A_MFAST = true;
    static constexpr bool B_NFAST = false;   // W[co][ci*k*k]
    const float* A; float* C; const float* W; const float* bias; const int2* ktab;
    int M, N, K;          // M = rows*Ho*Wo, N = Co, K = Ci*k*k
    int Ho, Wo, Hi, Wi, ldA, ldC, s, p;
    int acc;
    ConeClip clip;   // clip.rows null: none
    struct MCtx { long base, cbase; int iy, ix; bool ok, in; };
    __device__ MCtx mctx(int m) const {
        MCtx c;
        c.ok = m < M;
        int mm = c.ok ? m : 0;
        int per = Ho * Wo;
        int r = mm / per, rem = mm - r * per;
        int y = rem / Wo, x = rem - y * Wo;
        c.iy = s * y - p;
        c.ix = s * x - p;
        c.base = (long)r * ldA + (long)c.iy * Wi + c.ix;
        c.cbase = (long)r * ldC + rem;
        c.in = true;
        if (clip.rows) {
            int oy, ox;
            cone_origin(clip, r, oy, ox);
            c.in = oy + y >= 0 && oy + y < clip.H && ox + x >= 0 && ox + x < clip.W;
        }
        return c;
    }
    __device__ float a(const MCtx& c, int k) const {
        if (!c.ok || k >= K) return 0.f;
        int2 t = ktab[k];
        int ky = t.y >> 16, kx = t.y & 0xffff;
        int y = c.iy + ky, x = c.ix + kx;
        if ((unsigned)y >= (unsigned)Hi || (unsigned)x >= (unsigned)Wi) return 0.f;
        return A[c.base + t.x];
    }
    __device__ float b(int k, int n) const { return (k < K && n < N) ? W[(long)n * K + k] : 0.f; }
    // A elements of one K-tile within a single tap (Ci % 16 == 0); K ordered (ci / 16, ky, kx,
    // ci % 16): the k-tiles of one 16-channel group are its taps, one after the other
    int tile_ok, Ci, kw, HiWi;
    template <int NA>
    __device__ void a_tile(const MCtx& c, int k0, const int* ks, float* out) const {
        const int kt = k0 >> 4;
        const int cg = kt / (kw * kw), tap = kt - cg * kw * kw;
        const int ky = tap / kw, kx = tap - ky * kw;
        const int ci0 = cg * 16 + (k0 & 15);   // k0 carries the thread's first k within the tile
        const int y = c.iy + ky, x = c.ix + kx;
        const bool ok = c.ok && k0 < K && (unsigned)y < (unsigned)Hi && (unsigned)x < (unsigned)Wi;
        const float* src = A + (c.base + (long)ci0 * HiWi + ky * Wi + kx);
#pragma unroll
        for (int i = 0; i < NA; ++i) out[i] = ok ? src[(long)ks[i] * HiWi] : 0.f;
    }
    __device__ void store_ctx(const MCtx& c, int n, float v) const {
        if (c.ok && n < N) {
            float* q = C + c.cbase + (long)n * Ho * Wo;
            v = c.in ? v + bias[n] : 0.f;
            *q = acc ? *q + v : v;
        }
    }
};

// ------------------------------------------------------------------ kernel
template <int BM, int BN, int WAVES_M, class P>
__global__ __launch_bounds__(256) void k_gemm(P p) {
    constexpr int WAVES_N = 4 / WAVES_M;
    constexpr int WTM = BM / WAVES_M, WTN = BN / WAVES_N;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    constexpr int APAD = (16 - (BM % 32) + 32) % 32;   // row stride = 16 mod 32 banks
    constexpr int BPAD = (16 - (BN % 32) + 32) % 32;
    constexpr int LDA_S = BM + APAD, LDB_S = BN + BPAD;
    constexpr int A_PER = BM * BK / 256, B_PER = BN * BK / 256;
    static_assert(A_PER >= 1 && B_PER >= 1, "tile too small");
    __shared__ float As[2][BK][LDA_S];
    __shared__ float Bs[2][BK][LDB_S];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WAVES_M, wn = wave / WAVES_M;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int nk = (p.K + BK - 1) / BK;

    // A element map: either m-fast (gathers along positions) or k-fast (row-major rows)
    int a_m[A_PER > 0 ? (P::A_MFAST ? 1 : A_PER) : 1];
    int a_k[A_PER];
    typename P::MCtx actx[P::A_MFAST ? 1 : A_PER];
    if (P::A_MFAST) {
        constexpr int KSTEP = 256 / BM;
        a_m[0] = tid % BM;
        for (int i = 0; i < A_PER; ++i) a_k[i] = tid / BM + i * KSTEP;
        actx[0] = p.mctx(m0 + a_m[0]);
    } else {
        for (int i = 0; i < A_PER; ++i) {
            a_k[i] = tid % BK;
            a_m[i] = tid / BK + i * (256 / BK);
            actx[i] = p.mctx(m0 + a_m[i]);
        }
    }
    int b_k[B_PER], b_n[B_PER];
    for (int i = 0; i < B_PER; ++i) {
        if (P::B_NFAST) {
            constexpr int KSTEP = 256 / BN;
            b_n[i] = tid % BN;
            b_k[i] = tid / BN + i * KSTEP;
        } else {
            b_k[i] = tid % BK;
            b_n[i] = tid / BK + i * (256 / BK);
        }
    }

    float ra[A_PER], rb[B_PER];
    auto load = [&](int kt) {
        const int k0 = kt * BK;
        if (P::A_MFAST && p.tile_ok) {
            int kofs[A_PER];
#pragma unroll
            for (int i = 0; i < A_PER; ++i) kofs[i] = a_k[i] - a_k[0];
            p.template a_tile<A_PER>(actx[0], k0 + a_k[0], kofs, ra);
        } else {
            for (int i = 0; i < A_PER; ++i)
                ra[i] = p.a(actx[P::A_MFAST ? 0 : i], k0 + a_k[i]);
        }
        for (int i = 0; i < B_PER; ++i) rb[i] = p.b(k0 + b_k[i], n0 + b_n[i]);
    };
    auto stash = [&](int buf) {
        for (int i = 0; i < A_PER; ++i) As[buf][a_k[i]][P::A_MFAST ? a_m[0] : a_m[i]] = ra[i];
        for (int i = 0; i < B_PER; ++i) Bs[buf][b_k[i]][b_n[i]] = rb[i];
    };

    floatx4 acc[FM][FN];
    for (int i = 0; i < FM; ++i)
        for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    if (nk > 0) {
        load(0);
        stash(0);
        __syncthreads();
    }
    const int lrow = lane & 15, lk = lane >> 4;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load(kt + 1);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float fa[FM], fb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) fa[i] = As[cur][kk + lk][wm * WTM + i * 16 + lrow];
#pragma unroll
            for (int j = 0; j < FN; ++j) fb[j] = Bs[cur][kk + lk][wn * WTN + j * 16 + lrow];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) stash(cur ^ 1);
        __syncthreads();
    }

    // D layout of 16x16x4: lane holds rows 4*(lane/16) + v, column lane%16.
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = m0 + wm * WTM + i * 16 + 4 * lk + v;
            const auto c = p.mctx(m);
#pragma unroll
            for (int j = 0; j < FN; ++j) p.store_ctx(c, n0 + wn * WTN + j * 16 + lrow, acc[i][j][v]);
        }
    }
}

template <class P>
static void run_gemm(const P& p, hipStream_t st) {
    dim3 blk(256);
    // tile shape only changes how outputs are grouped into workgroups, never the order in
    // which an output element accumulates over K, so it may follow the grid size
    const long big = (long)cdiv(p.M, 128) * cdiv(p.N, 128);
    if (p.N > 64 && big < 512) {
        dim3 grid(cdiv(p.M, 64), cdiv(p.N, 64));
        hipLaunchKernelGGL((k_gemm<64, 64, 2, P>), grid, blk, 0, st, p);
        MNB_HIP(hipGetLastError());
        return;
    }
    if (p.N <= 16) {
        dim3 grid(cdiv(p.M, 256), cdiv(p.N, 16));
        hipLaunchKernelGGL((k_gemm<256, 16, 4, P>), grid, blk, 0, st, p);
    } else if (p.N <= 32) {
        dim3 grid(cdiv(p.M, 128), cdiv(p.N, 32));
        hipLaunchKernelGGL((k_gemm<128, 32, 4, P>), grid, blk, 0, st, p);
    } else if (p.N <= 64) {
        dim3 grid(cdiv(p.M, 128), cdiv(p.N, 64));
        hipLaunchKernelGGL((k_gemm<128, 64, 2, P>), grid, blk, 0, st, p);
    } else {
        dim3 grid(cdiv(p.M, 128), cdiv(p.N, 128));
        hipLaunchKernelGGL((k_gemm<128, 128, 2, P>), grid, blk, 0, st, p);
    }
    MNB_HIP(hipGetLastError());
}

void launch_fc_backsub(const float* A, const float* W, float* C, int M, int dout, int din,
                       bool accumulate, hipStream_t st) {
    if (M <= 0) return;
    FcBack p;
    p.A = A; p.W = W; p.C = C; p.M = M; p.N = din; p.K = dout; p.acc = accumulate;
    run_gemm(p, st);
}

void launch_fc_forward(const float* G, const float* W, const float* b, float* C, int M, int din,
                       int dout, bool accumulate, hipStream_t st) {
    if (M <= 0) return;
    FcFwd p;
    p.A = G; p.W = W; p.bias = b; p.C = C; p.M = M; p.N = dout; p.K = din; p.acc = accumulate;
    run_gemm(p, st);
}

// ------------------------------------------------------------------ small-Ci transposed conv (VALU)
// For layers whose input has very few channels (Ci < 16) an MFMA tile would be
// mostly padding; these layers are HBM-bound, so one thread per output element
// gathers its taps directly.
__global__ __launch_bounds__(256) void k_convT_valu(const float* __restrict__ A, float* __restrict__ C,
                                                   const float* __restrict__ W, int M, int Ci, int Hi,
                                                   int Wi, int Co, int Ho, int Wo, int k, int s, int p,
                                                   int acc) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long per = (long)Ci * Hi * Wi;
    if (idx >= (long)M * per) return;
    int r = (int)(idx / per);
    int rem = (int)(idx - (long)r * per);
    int ci = rem / (Hi * Wi);
    int pos = rem - ci * Hi * Wi;
    int Y = pos / Wi, X = pos - Y * Wi;
    const float* Ar = A + (long)r * Co * Ho * Wo;
    float sum = 0.f;
    for (int ky = (Y + p) % s; ky < k; ky += s) {
        int y = (Y + p - ky) / s;
        if (y < 0 || y >= Ho) continue;
        for (int kx = (X + p) % s; kx < k; kx += s) {
            int x = (X + p - kx) / s;
            if (x < 0 || x >= Wo) continue;
            const float* w = W + ((long)ci * k + ky) * k + kx;
            const float* a = Ar + (long)y * Wo + x;
            for (int co = 0; co < Co; ++co) sum += a[(long)co * Ho * Wo] * w[(long)co * Ci * k * k];
        }
    }
    float* out = C + idx;
    *out = acc ? *out + sum : sum;
}

// Transposed convolution into very few channels (Ci <= 4, the first layer of CIFAR
// networks): one workgroup per (row, 16x16 output tile) stages the coefficient window the
// tile depends on, 8 output channels of the layer at a time, into LDS; each thread owns one
// output pixel and accumulates all Ci input channels, so every coefficient is read once from
// global memory per tile and reused for all taps and channels from LDS.
constexpr int TCT = 16;     // output tile edge
constexpr int TCO = 8;      // layer output channels staged per step
template <int CI>
__global__ __launch_bounds__(256) void k_convT_small(const float* __restrict__ A, float* __restrict__ C,
                                                     const float* __restrict__ W, int Hi, int Wi, int Co,
                                                     int Ho, int Wo, int k, int s, int p, int acc, int tiles_x,
                                                     int WY, int WX) {
    extern __shared__ float sm[];
    float* s_w = sm;                       // [Co][CI][k][k]
    float* s_a = sm + Co * CI * k * k;     // [TCO][WY][WX] coefficient window
    const int t = threadIdx.x;
    const int r = blockIdx.y;
    const int tile = blockIdx.x, ty0 = (tile / tiles_x) * TCT, tx0 = (tile % tiles_x) * TCT;
    const int Y = ty0 + t / TCT, X = tx0 + t % TCT;
    // window origin on the layer output: smallest y that any pixel of the tile reaches
    const int y0 = (ty0 + p - (k - 1)) >= 0 ? (ty0 + p - (k - 1)) / s : -((-(ty0 + p - (k - 1)) + s - 1) / s);
    const int x0 = (tx0 + p - (k - 1)) >= 0 ? (tx0 + p - (k - 1)) / s : -((-(tx0 + p - (k - 1)) + s - 1) / s);
    for (int i = t; i < Co * CI * k * k; i += 256) s_w[i] = W[i];
    const float* Ar = A + (long)r * Co * Ho * Wo;
    float out[CI];
#pragma unroll
    for (int c = 0; c < CI; ++c) out[c] = 0.f;
    const int HoWo = Ho * Wo, win = WY * WX;
    for (int c0 = 0; c0 < Co; c0 += TCO) {
        const int nco = Co - c0 < TCO ? Co - c0 : TCO;
        __syncthreads();   // previous window consumed (and weights visible on the first pass)
        for (int i = t; i < nco * win; i += 256) {
            const int co = i / win, rem = i - co * win, wy = rem / WX, wx = rem - wy * WX;
            const int y = y0 + wy, x = x0 + wx;
            s_a[i] = (y >= 0 && y < Ho && x >= 0 && x < Wo) ? Ar[(long)(c0 + co) * HoWo + y * Wo + x] : 0.f;
        }
        __syncthreads();
        if (Y < Hi && X < Wi) {
            const int Yp = Y + p, Xp = X + p;
            for (int ky = Yp % s; ky < k; ky += s) {
                const int wy = (Yp - ky) / s - y0;
                for (int kx = Xp % s; kx < k; kx += s) {
                    const int wx = (Xp - kx) / s - x0;
                    const float* ap = s_a + wy * WX + wx;
                    const float* wp = s_w + ((long)c0 * CI * k + ky) * k + kx;   // [co][ci][ky][kx]
                    for (int co = 0; co < nco; ++co) {
                        const float av = ap[co * win];
#pragma unroll
                        for (int c = 0; c < CI; ++c) out[c] += av * wp[(co * CI + c) * k * k];
                    }
                }
            }
        }
    }
    if (Y < Hi && X < Wi) {
        float* Cr = C + (long)r * CI * Hi * Wi + Y * Wi + X;
#pragma unroll
        for (int c = 0; c < CI; ++c) {
            float* q = Cr + (long)c * Hi * Wi;
            *q = acc ? *q + out[c] : out[c];
        }
    }
}

static bool launch_convT_small(const ConvGeom& g, const float* A, float* C, int M, bool accumulate, hipStream_t st) {
    if (g.Ci > 4 || g.k > 5 || g.s > 2) return false;
    const int tiles_y = cdiv(g.Hi, TCT), tiles_x = cdiv(g.Wi, TCT);
    // window rows: y from ceil((ty0 + p - (k-1)) / s) to (ty0 + TCT - 1 + p) / s
    const int WY = (TCT - 1 + g.k - 1) / g.s + 2, WX = WY;
    const size_t lds = ((size_t)g.Co * g.Ci * g.k * g.k + (size_t)TCO * WY * WX) * sizeof(float);
    if (lds > 64 * 1024) return false;
    // rows go on grid.y (at most 65535 per launch): larger batches are launched in row slices
    const long ldA = (long)g.Co * g.Ho * g.Wo, ldC = (long)g.Ci * g.Hi * g.Wi;
    for (int r0 = 0; r0 < M; r0 += kMaxGridY) {
        const int nr = M - r0 < kMaxGridY ? M - r0 : kMaxGridY;
        const dim3 grid(tiles_y * tiles_x, nr);
        const float* Ar = A + r0 * ldA;
        float* Cr = C + r0 * ldC;
        switch (g.Ci) {
            case 1: hipLaunchKernelGGL(k_convT_small<1>, grid, dim3(256), lds, st, Ar, Cr, g.W, g.Hi, g.Wi, g.Co,
                                       g.Ho, g.Wo, g.k, g.s, g.p, (int)accumulate, tiles_x, WY, WX); break;
            case 2: hipLaunchKernelGGL(k_convT_small<2>, grid, dim3(256), lds, st, Ar, Cr, g.W, g.Hi, g.Wi, g.Co,
                                       g.Ho, g.Wo, g.k, g.s, g.p, (int)accumulate, tiles_x, WY, WX); break;
            case 3: hipLaunchKernelGGL(k_convT_small<3>, grid, dim3(256), lds, st, Ar, Cr, g.W, g.Hi, g.Wi, g.Co,
                                       g.Ho, g.Wo, g.k, g.s, g.p, (int)accumulate, tiles_x, WY, WX); break;
            default: hipLaunchKernelGGL(k_convT_small<4>, grid, dim3(256), lds, st, Ar, Cr, g.W, g.Hi, g.Wi, g.Co,
                                        g.Ho, g.Wo, g.k, g.s, g.p, (int)accumulate, tiles_x, WY, WX); break;
        }
        MNB_HIP(hipGetLastError());
    }
    return true;
}

void launch_conv_backsub(const ConvGeom& g, const float* A, float* C, int M, bool accumulate,
                         hipStream_t st) {
    if (M <= 0) return;
    if (launch_conv_backsub_rows(g, A, C, M, accumulate, st)) return;
    if (launch_convT_first(g, A, C, M, accumulate, st)) return;
    if (launch_convT_small(g, A, C, M, accumulate, st)) return;
    if (g.Ci < 16) {
        long total = (long)M * g.Ci * g.Hi * g.Wi;
        hipLaunchKernelGGL(k_convT_valu, dim3(cdiv(total, 256)), dim3(256), 0, st, A, C, g.W, M, g.Ci,
                           g.Hi, g.Wi, g.Co, g.Ho, g.Wo, g.k, g.s, g.p, (int)accumulate);
        MNB_HIP(hipGetLastError());
        return;
    }
    if (launch_conv_backsub_win(g, A, C, M, accumulate, st)) return;
    for (int f = 0; f < g.n_phase; ++f) {
        const ConvPhase& ph = g.ph[f];
        if (ph.nY <= 0 || ph.nX <= 0) continue;
        ConvBack p;
        p.A = A; p.C = C; p.ktab = ph.ktab;
        p.M = M * ph.nY * ph.nX; p.N = g.Ci; p.K = g.Co * ph.Ty * ph.Tx;
        p.nY = ph.nY; p.nX = ph.nX; p.Ho = g.Ho; p.Wo = g.Wo;
        p.ldA = g.Co * g.Ho * g.Wo; p.ldC = g.Ci * g.Hi * g.Wi; p.HiWi = g.Hi * g.Wi; p.Wi = g.Wi;
        p.Y0 = ph.Y0; p.X0 = ph.X0; p.s = g.s; p.q0y = ph.q0y; p.q0x = ph.q0x;
        p.acc = accumulate;
        p.Co = g.Co; p.Tx = ph.Tx; p.Ty = ph.Ty; p.HoWo = g.Ho * g.Wo;
        p.tile_ok = (g.Co % BK) == 0 && ph.Wpg != nullptr;
        p.Wp = p.tile_ok ? ph.Wpg : ph.Wp;
        run_gemm(p, st);
    }
}

void launch_conv_forward(const ConvGeom& g, const float* G, float* C, int M, bool accumulate,
                         hipStream_t st, const ConeClip* clip) {
    if (M <= 0) return;
    // the row-resident kernels write no clip
    if (!clip && launch_conv_forward_rows(g, G, C, M, accumulate, st)) return;
    if (launch_conv_first(g, G, C, M, accumulate, st, clip)) return;
    if (launch_conv_forward_win(g, G, C, M, accumulate, st, clip)) return;
    ConvFwd p;
    p.clip = clip ? *clip : ConeClip{};
    p.A = G; p.C = C; p.bias = g.b; p.ktab = g.fwd_ktab;
    p.Ci = g.Ci; p.kw = g.k; p.HiWi = g.Hi * g.Wi;
    p.tile_ok = (g.Ci % BK) == 0 && g.Wg != nullptr;
    p.W = p.tile_ok ? g.Wg : g.Wf;
    p.M = M * g.Ho * g.Wo; p.N = g.Co; p.K = g.Ci * g.k * g.k;
    p.Ho = g.Ho; p.Wo = g.Wo; p.Hi = g.Hi; p.Wi = g.Wi;
    p.ldA = g.Ci * g.Hi * g.Wi; p.ldC = g.Co * g.Ho * g.Wo; p.s = g.s; p.p = g.p;
    p.acc = accumulate;
    run_gemm(p, st);
}

}  // namespace mnb
