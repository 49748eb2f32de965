// Fused bottom of a back-substitution pass on v_mfma_f32_16x16x4_f32, for networks
// whose first layer is a convolution into 16 channels with at most 32 taps per
// channel (ConvSmall, the ResNet stems).
//
// One workgroup owns one chunk of rows of one instance (subproblem, parameter
// set).  The positions of ReLU layer 0 are cut into 16-position tiles; each of the
// 16 wavefronts owns one tile (TPW), and in a tile lane (lr, lk) owns the four
// neurons (channel 4 lk + v, position 16 mt + lr), v = 0..3, for the whole chunk.
// Per row:
//   fold of ReLU layer 0 (Eq. 5) in registers: a' -> ahat
//   transposed first convolution (Eq. 2): T[pos][tap] = sum_co ahat[co][pos] W[co][tap],
//       with ahat as the MFMA A operand straight from registers    -> T in LDS
//   barrier; col2im of T, concretisation over the box (Eq. 6), x*   -> x* in LDS
//   block reduction of the bound (barrier; the last wavefront finishes the sums and
//       stores the bounds)
//   adjoint: ghat^T[co][pos] = sum_tap W[co][tap] x*[pos][tap] + b, whose MFMA
//       output lands in the lanes that hold a' for the same neurons, so the
//       relaxation of ReLU layer 0, the alpha-gradient sums and the rows' g are
//       computed in registers.
// Rows are taken two at a time where registers allow (RP), with two barriers per
// iteration; the next rows' coefficients are loaded an iteration ahead (into LDS with
// one input element per thread).  The alpha sums run over the chunk's rows in order;
// the ghat sums for beta come from per-element counts of x* = hi (k_bottom_reduce).
#include "bottom.h"
#include "../../include/mnbab.h"

namespace mnb {

namespace {

constexpr int MBT = 1024;        // threads (16 wavefronts, one 16-position tile each)
constexpr int MNW = MBT / 64;
static_assert(BOTTOM_CHUNK_ROWS <= 2 * MNW, "the prologue reads two rows per wavefront");
typedef float f4 __attribute__((ext_vector_type(4)));

// One dword per lane from global memory straight into LDS (global_load_lds_dword): lane l's
// value lands at byte lds + 4 l of LDS; lds must be wave-uniform.  Written as asm so that the
// compiler, which otherwise makes every later LDS access and barrier wait for such loads,
// does not track it: the load has no destination register, only the issuing wavefront reads
// what it writes, and it does so after mf_drain().  M0 (the LDS base of the load) is not used
// by any compiler-generated code of this kernel.
__device__ __forceinline__ void load_to_lds(const float* g, const float* lds) {
    const unsigned la = (unsigned)(size_t)lds;
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dword %0, off" ::"v"(g), "s"(la) : "memory");
}

// Every load and store of this wavefront complete (vmcnt 0), loads into LDS included; no memory
// access moves across it.
__device__ __forceinline__ void mf_drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Workgroup barrier for LDS data: this wavefront's LDS instructions are complete before the
// barrier.  Unlike a release fence, it does not wait for the wavefront's loads into LDS
// (s_pf), which only that wavefront reads, after its own vmcnt drain.
__device__ __forceinline__ void lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Sum of three per-thread values over the block (fixed order), valid in thread 0 only;
// one barrier.
__device__ __forceinline__ void bsum3(float& x, float& y, float& z, float (*red)[MNW]) {
    x = wave_sum(x);
    y = wave_sum(y);
    z = wave_sum(z);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = x;
        red[1][w] = y;
        red[2][w] = z;
    }
    lds_sync();
    if (threadIdx.x != 0) return;
    float v[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float* rq = red[q];
        const float h0 = ((rq[0] + rq[1]) + (rq[2] + rq[3])) + ((rq[4] + rq[5]) + (rq[6] + rq[7]));
        const float h1 = ((rq[8] + rq[9]) + (rq[10] + rq[11])) + ((rq[12] + rq[13]) + (rq[14] + rq[15]));
        v[q] = h0 + h1;
    }
    x = v[0];
    y = v[1];
    z = v[2];
}

// Taps of the first convolution that reach one input element (at most 3 x 3 with a runtime shape).
constexpr int nto_taps(int KK, int SS) { return KK ? ((KK + SS - 1) / SS) * ((KK + SS - 1) / SS) : 9; }
// Rows per iteration: two for first layers of at most 16 taps with a compile-time shape.
constexpr int mf_rows(int KK, int NTT) { return (NTT == 1 && KK != 0) ? 2 : 1; }
// Per-thread index tables in LDS (one input element per thread, 4 taps and 4 adjoint steps).
constexpr bool mf_tab(bool O1, int KK, int SS, int NTT) { return O1 && nto_taps(KK, SS) == 4 && NTT == 1; }
// Next rows prefetched straight into LDS: with one input element per thread (no global loads
// left in the row loop that would wait behind them) and rows read from A.
constexpr bool mf_pf_lds(bool SRC1, bool O1) { return O1 && !SRC1; }

// KK, SS: kernel size and stride as constants (0: runtime); NTT: 16-tap tiles of the first
// convolution (1: at most 16 taps, 2: at most 32); SRC1: rows built from the objective
// convolution's filter; O1: at most one input element per thread (d0 <= 1024), whose col2im
// taps, box and x* count are then held in registers for the whole chunk.
// Rows are taken two at a time (RP, for first layers of at most 16 taps with a compile-time
// shape): the barriers, block sums and memory drain of an iteration serve both, and their
// MFMA chains interleave.
template <int TPW, int KK, int SS, int NTT, bool SRC1, bool O1>
__global__ __launch_bounds__(MBT) void k_bottom_mf(BottomArgs a) {
    static_assert(TPW == 1, "one tile per wavefront");
    constexpr int RP = mf_rows(KK, NTT);   // rows per iteration (registers permitting)
    constexpr bool PFL = mf_pf_lds(SRC1, O1);   // next rows prefetched into LDS (else registers)
    constexpr int KSM = 4 * NTT;   // 4-tap steps of the adjoint product
    const int k = KK ? KK : a.k;
    const int s = SS ? SS : a.s;
    const int d1 = a.d1, d0 = a.d0;
    const int HoWo = a.Ho * a.Wo, HiWi = a.Hi * a.Wi;
    const int kk = k * k, ntap = a.Ci * kk;
    const int MT = (HoWo + 15) >> 4;
    // tap products T[tap][pos]: per tap a stride of HP = 16 MT + 1 positions; position 16 MT of
    // tap 0 is never written and holds zero (the target of col2im taps that do not exist)
    const int HP = 16 * MT + 1, TZ = 16 * MT;
    const int TSZ = 16 * NTT * HP;
    const int XS = d0 + 1;   // x* rows: d0 elements and a zero (the target of absent adjoint taps)
    extern __shared__ float4 smem4[];
    float4* s_rx = smem4;                                // [d1] relaxation {a' >= 0 slope, a' < 0 slope, intercept, add}
    float* smem = reinterpret_cast<float*>(smem4 + d1);
    float* s_T = smem;                                   // [RP][16 NTT][HP] tap products, tap-major
    float* s_x = s_T + RP * TSZ;                         // [RP][XS] x* of the current rows
    int* s_xc = reinterpret_cast<int*>(s_x + RP * XS);   // [d0] rows of the chunk with x*_o = hi_o (!O1)
    float* s_lo = s_x + RP * XS + d0;                    // [d0] box (box_lds)
    float* s_hi = s_lo + d0;                             // [d0]
    float* s_sg = s_x + RP * XS + d0 + (a.box_lds ? 2 * d0 : 0);   // [d1] sum of g (MNC only)
    // per thread, row-invariant index tables (NTO == 4, KSM == 4): col2im taps and adjoint gathers
    constexpr bool TAB = mf_tab(O1, KK, SS, NTT);
    const int tab_off = (int)((s_sg + (a.gsum_out ? d1 : 0)) - reinterpret_cast<float*>(smem4));
    int4* s_tab = reinterpret_cast<int4*>(smem4) + (tab_off + 3) / 4;   // [2][MBT] (TAB)
    __shared__ float red[3 * RP][MNW];
    __shared__ RowDesc s_rd[BOTTOM_CHUNK_ROWS];
    __shared__ float s_crow[BOTTOM_CHUNK_ROWS];
    __shared__ float s_old[BOTTOM_CHUNK_ROWS];
    // next rows' coefficients, per wavefront [b][v][lane] (a separate array, so that the
    // compiler sees that no other LDS access touches what the loads into LDS write)
    __shared__ float s_pf[PFL ? MNW * RP * 256 : 1];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
    // The prologue's loads are issued in four dependent levels, each level's loads in flight
    // together: chunk -> instance -> (the chunk's rows, query, relaxation inputs, first
    // coefficients) -> (box, the rows' previous bounds).  Only one workgroup fits on a CU, so
    // nothing else hides this latency.
    const int ib = a.cinst[blockIdx.x];
    const int cr0 = a.cr0[blockIdx.x];
    const int nr = min(a.cr1[blockIdx.x] - cr0, BOTTOM_CHUNK_ROWS);
    // first-layer weights as MFMA operands held for the whole chunk:
    // transposed product B[k = co][n = tap] with co = 4 lk + ks, tap = 16 nt + lr;
    // adjoint product A[m = co][k = tap] with co = lr, tap = 4 ks + lk
    float bT[NTT][4], aW[KSM];
#pragma unroll
    for (int nt = 0; nt < NTT; ++nt)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int tap = nt * 16 + lr;
            bT[nt][ks] = tap < ntap ? a.W1[(4 * lk + ks) * ntap + tap] : 0.f;
        }
#pragma unroll
    for (int ks = 0; ks < KSM; ++ks) {
        const int tap = 4 * ks + lk;
        aW[ks] = tap < ntap ? a.W1[lr * ntap + tap] : 0.f;
    }
    // bias of the first convolution (16 channels; lane group lk owns channels 4 lk .. 4 lk + 3),
    // read from LDS where used
    __shared__ float4 s_b1[4];
    if (t < 16) reinterpret_cast<float*>(s_b1)[t] = a.b1[t];
    const InstDesc in = a.inst[ib];

    // owned neurons: tile mt = wave, neuron (co = 4 lk + v, pos = 16 mt + lr)
    const int mt = wave;
    const int pos = mt * 16 + lr;
    const bool pv = pos < HoWo;
    // the chunk's rows (at most BOTTOM_CHUNK_ROWS = 2 MNW by construction of the chunks):
    // descriptor, constant and the first 64 constant partials of rows wave and wave + MNW
    // (wave-uniform row index, so the descriptors come through scalar loads)
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    RowDesc rdq[2];
    float crq[2] = {0.f, 0.f}, cpq[2] = {0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int ri = wv + q * MNW;
        if (ri < nr) {
            const long r = cr0 + ri;
            rdq[q] = a.rows[r];
            if constexpr (!SRC1) {
                crq[q] = a.c[r];
                if (lane < a.ncp) cpq[q] = a.cpart[r * a.ldcp + lane];
            }
        }
    }
    const int qv = a.qid[in.slot];
    // relaxation inputs of the owned neurons (all loaded, used by case below)
    const long so0 = (long)in.slot * a.ld_state;
    const long po0 = ((long)in.slot * a.n_sets + in.set) * a.ld_param;
    float rl[4], ru[4], ral[4], rbe[4], rvh[4];
    int rs[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int j = (4 * lk + v) * HoWo + pos;
        rl[v] = ru[v] = ral[v] = rbe[v] = rvh[v] = 0.f;
        rs[v] = 0;
        if (pv) {
            rl[v] = a.l[so0 + j];
            ru[v] = a.u[so0 + j];
            rs[v] = (int)a.S[so0 + j];
            ral[v] = a.alpha[po0 + j];
            rbe[v] = a.beta[po0 + j];
            if (a.vhat) rvh[v] = a.vhat[(long)ib * d1 + j];
        }
    }
    // coefficients of the next rows, loaded one iteration ahead (the first ones before the
    // barrier that ends the prologue): with PFL straight into the wavefront's LDS slots
    // s_pf[wave][b][v][lane], otherwise into registers.  Every lane loads, so that no load sits
    // in a branch: lanes without a position read position 0 of their channel and rows past the
    // chunk's end the chunk's last row; neither value reaches a result, since a lane without a
    // position has a zero relaxation and a row past the end is neither summed nor stored.
    const int pc = pv ? pos : 0;
    float* pfw = s_pf + (PFL ? wv * (RP * 256) : 0);
    // wavefronts without a position tile (16 tiles for ConvSmall's 11) take no LDS prefetch: their
    // coefficients are zero (they feed no MFMA and no store)
    const bool pfw_on = wv < MT;
    float nx[PFL || SRC1 ? 1 : RP][4];
    if constexpr (!SRC1) {
        if (nr > 0) {
#pragma unroll
            for (int b = 0; b < RP; ++b) {
                const float* rowp = a.A + (long)(cr0 + min(b, nr - 1)) * d1;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if constexpr (PFL) {
                        if (pfw_on) load_to_lds(rowp + (4 * lk + v) * HoWo + pc, pfw + (b * 4 + v) * 64);
                    } else {
                        nx[b][v] = rowp[(4 * lk + v) * HoWo + pc];
                    }
                }
            }
        }
    }
    // box: O1, the owned input element o = t; otherwise staged in LDS (box_lds)
    const float* glo = a.lo + (long)qv * d0;
    const float* ghi = a.hi + (long)qv * d0;
    float lo_o = 0.f, hi_o = 0.f;
    int xc_o = 0;   // O1: rows of the chunk with x*_o = hi_o for the owned element
    if constexpr (O1) {
        if (t < d0) {
            lo_o = glo[t];
            hi_o = ghi[t];
        }
    } else {
        for (int o = t; o < d0; o += MBT) {
            s_xc[o] = 0;
            if (a.box_lds) {
                s_lo[o] = glo[o];
                s_hi[o] = ghi[o];
            }
        }
    }
    // previous bound of each row: of its objective neuron (each (slot, neuron) of the objective
    // layer has exactly one row in a pass), or the best bound so far of a spec row
    float oldq[2] = {0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int ri = wv + q * MNW;
        if (ri < nr) {
            const RowDesc rd = rdq[q];
            if (a.mode == 0) {
                const long e = so0 + a.state_off_obj + rd.j;
                const float* src = rd.sign > 0 ? a.lw : a.uw;
                oldq[q] = src[e];
            } else if (a.mode == 1) {
                oldq[q] = a.best[cr0 + ri];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int ri = wv + q * MNW;
        if (ri < nr) {
            const RowDesc rd = rdq[q];
            float cr;
            if constexpr (SRC1) {
                cr = (float)rd.sign * a.bias_obj[rd.j];
            } else {
                // constant partials beyond the first 64 (rare), then the wave sum in lane order
                float sp = cpq[q];
                for (int kq = lane + 64; kq < a.ncp; kq += 64) sp += a.cpart[(long)(cr0 + ri) * a.ldcp + kq];
                cr = crq[q] + wave_sum(sp);
            }
            if (lane == 0) {
                s_rd[ri] = rd;
                s_crow[ri] = cr;
                s_old[ri] = oldq[q];
            }
        }
    }
    if (a.gsum_out)
        for (int j = t; j < d1; j += MBT) s_sg[j] = 0.f;
    if (t < RP) {
        s_T[t * TSZ + TZ] = 0.f;
        s_x[t * XS + d0] = 0.f;
    }

    // relaxation of ReLU layer 0 on the owned neurons (split first, then stable, then unstable)
    // to LDS: slope where a' >= 0, slope and intercept where a' < 0 (the intercept is > 0
    // exactly when unstable), S beta + (Phat^T gamma)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        if (!pv) continue;
        const float l = rl[v], uu = ru[v];
        const int sj = rs[v];
        float dp = 0.f, dn = 0.f, bn = 0.f;
        if (sj == -1) {
            dp = dn = 1.f;
        } else if (sj == 1) {
        } else if (l >= 0.f) {
            dp = dn = 1.f;
        } else if (uu <= 0.f) {
        } else {
            dp = ral[v];
            const float w = uu - l;
            dn = uu / w;
            bn = -(uu * l) / w;
        }
        const float ad = (sj != 0 ? (float)sj * rbe[v] : 0.f) + rvh[v];
        s_rx[(4 * lk + v) * HoWo + pos] = make_float4(dp, dn, bn, ad);
    }
    // O1: col2im taps of the owned input element (s_T offsets, TZ (a zero): none)
    constexpr int NTO = nto_taps(KK, SS);
    int tix[O1 ? NTO : 1];
    if constexpr (O1) {
        const bool ov = t < d0;
        const int o = ov ? t : 0;
        const int ci = o / HiWi, qq = o - ci * HiWi;
        const int Yq = qq / a.Wi;
        const int Yp = Yq + a.p, Xp = qq - Yq * a.Wi + a.p;
        const int nty = (k + s - 1) / s;
#pragma unroll
        for (int q = 0; q < NTO; ++q) {
            const int ty = q / (KK ? (KK + SS - 1) / SS : 3), tx = q - ty * (KK ? (KK + SS - 1) / SS : 3);
            const int ky = Yp % s + ty * s, kx = Xp % s + tx * s;
            const int y = (Yp - ky) / s, x = (Xp - kx) / s;
            const bool tv = ov && ty < nty && tx < nty && ky < k && kx < k && Yp >= ky && Xp >= kx && y < a.Ho && x < a.Wo;
            tix[q] = tv ? ((ci * k + ky) * k + kx) * HP + y * a.Wo + x : TZ;
        }
        if constexpr (TAB) s_tab[t] = make_int4(tix[0], tix[NTO > 1 ? 1 : 0], tix[NTO > 2 ? 2 : 0], tix[NTO > 3 ? 3 : 0]);
    }
    // adjoint B operand: s_x index of (pos, tap = 4 ks + lk), d0 (a zero): none
    int gidx[KSM];
    {
        const int y = pv ? pos / a.Wo : 0, x = pv ? pos - y * a.Wo : 0;
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks) {
            const int tap = 4 * ks + lk;
            int idx = d0;
            if (pv && tap < ntap) {
                const int ci = tap / kk, rr = tap - ci * kk, ky = rr / k, kx = rr - ky * k;
                const int Y = s * y - a.p + ky, X = s * x - a.p + kx;
                if ((unsigned)Y < (unsigned)a.Hi && (unsigned)X < (unsigned)a.Wi) idx = (ci * a.Hi + Y) * a.Wi + X;
            }
            gidx[ks] = idx;
        }
        if constexpr (TAB) s_tab[MBT + t] = make_int4(gidx[0], gidx[KSM > 1 ? 1 : 0], gidx[KSM > 2 ? 2 : 0], gidx[KSM > 3 ? 3 : 0]);
    }
    // (read at an in-bounds index by every lane, then zero for lanes without a position)
    auto relax = [&](int v) -> float4 {
        const float4 r = s_rx[(4 * lk + v) * HoWo + pc];
        return pv ? r : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    float da[4] = {0.f, 0.f, 0.f, 0.f};
    const float* vrow = a.v ? a.v + (long)ib * d1 : nullptr;
    const float gpv = a.gp ? a.gp[ib] : 0.f;
    // every prologue load complete, in a form the compiler sees (the loop issues no loads it
    // tracks, so it then places no waits inside the loop)
    vmem_drain();
    __syncthreads();

    for (int ri = 0; ri < nr; ri += RP) {
        const int nb = min(RP, nr - ri);   // rows this iteration (the second may be absent)
        // ---- row coefficients a on the owned neurons of ReLU layer 0
        // the relaxation of the owned neurons, read together with the prefetched rows below
        float4 rxq[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) rxq[v] = relax(v);
        float ap[RP][4];
        if constexpr (!SRC1) {
            if constexpr (PFL) {
                if (pfw_on) {
#pragma unroll
                    for (int b = 0; b < RP; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v) ap[b][v] = pfw[(b * 4 + v) * 64 + lane];
                } else {
#pragma unroll
                    for (int b = 0; b < RP; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v) ap[b][v] = 0.f;
                }
            } else {
#pragma unroll
                for (int b = 0; b < RP; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) ap[b][v] = nx[b][v];
            }
            if (ri + RP < nr) {
                // the slots are read before they are reloaded
                if constexpr (PFL) __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
#pragma unroll
                for (int b = 0; b < RP; ++b) {
                    const float* rowp = a.A + (long)(cr0 + min(ri + RP + b, nr - 1)) * d1;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if constexpr (PFL) {
                            if (pfw_on) load_to_lds(rowp + (4 * lk + v) * HoWo + pc, pfw + (b * 4 + v) * 64);
                        } else {
                            nx[PFL ? 0 : b][v] = rowp[(4 * lk + v) * HoWo + pc];
                        }
                    }
                }
                // register prefetch: keep the loads here, a full iteration ahead of their use
                // (the compiler would otherwise sink them next to it)
                if constexpr (!PFL) asm volatile("" ::: "memory");
            }
        } else {
            // +-e_j on the output of the objective convolution: its filter placed at j
#pragma unroll
            for (int b = 0; b < RP; ++b) {
                const RowDesc rd = s_rd[min(ri + b, nr - 1)];
                const float sgn = b < nb ? (float)rd.sign : 0.f;
                const int per = a.oHo * a.oWo;
                const int oco = rd.j / per, opos = rd.j - oco * per;
                const int oy = opos / a.oWo, ox = opos - oy * a.oWo;
                const float* wrow = a.Wobj + (long)oco * a.oCi * a.ok * a.ok;
                const int Y = pv ? pos / a.oWi : 0, X = pos - Y * a.oWi;
                const int ky = Y - a.os * oy + a.op, kx = X - a.os * ox + a.op;
                const bool in_w = pv && (unsigned)ky < (unsigned)a.ok && (unsigned)kx < (unsigned)a.ok;
#pragma unroll
                for (int v = 0; v < 4; ++v) ap[b][v] = in_w ? sgn * wrow[((4 * lk + v) * a.ok + ky) * a.ok + kx] : 0.f;
            }
        }
        if (vrow) {
            float vv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) vv[v] = pv ? vrow[(4 * lk + v) * HoWo + pos] : 0.f;
#pragma unroll
            for (int b = 0; b < RP; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) ap[b][v] += b < nb ? vv[v] : 0.f;
        }
        // ---- fold of ReLU layer 0 and the transposed first convolution of the owned tile
        float cpt[RP];
        {
            float ah[RP][4];
            const float4 b1q = s_b1[lk];
            const float b1g[4] = {b1q.x, b1q.y, b1q.z, b1q.w};
#pragma unroll
            for (int b = 0; b < RP; ++b) cpt[b] = 0.f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float4 rx = rxq[v];
#pragma unroll
                for (int b = 0; b < RP; ++b) {
                    const float p = ap[b][v];
                    const bool neg = p < 0.f;
                    ah[b][v] = p * (neg ? rx.y : rx.x) + (b < nb ? rx.w : 0.f);
                    cpt[b] += (neg ? p * rx.z : 0.f) + ah[b][v] * b1g[v];
                }
            }
            if (mt < MT) {
#pragma unroll
                for (int nt = 0; nt < NTT; ++nt) {
                    f4 acc[RP];
#pragma unroll
                    for (int b = 0; b < RP; ++b) acc[b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                        for (int b = 0; b < RP; ++b)
                            acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[b][ks], bT[nt][ks], acc[b], 0, 0, 0);
                    // lane holds T[pos = 16 mt + 4 lk + v][tap = 16 nt + lr]
#pragma unroll
                    for (int b = 0; b < RP; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int p2 = mt * 16 + 4 * lk + v;
                            s_T[b * TSZ + (nt * 16 + lr) * HP + p2] = acc[b][v];
                        }
                }
            }
        }
        if (a.Ap_out && pv) {
#pragma unroll
            for (int b = 0; b < RP; ++b)
                if (b < nb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) a.Ap_out[(long)(cr0 + ri + b) * d1 + (4 * lk + v) * HoWo + pos] = ap[b][v];
        }
        if (t == 0)
#pragma unroll
            for (int b = 0; b < RP; ++b) cpt[b] += b < nb ? s_crow[ri + b] - gpv : 0.f;
        // the owned element's col2im taps (written once in the prologue), read before the barrier
        int4 tv;
        if constexpr (TAB) tv = s_tab[t];
        lds_sync();
        // ---- col2im onto the input and concretisation over the box (Eq. 6), x*
        float lbp[RP], mag[RP];
#pragma unroll
        for (int b = 0; b < RP; ++b) lbp[b] = mag[b] = 0.f;
        if constexpr (O1) {
            if (t < d0) {
                int tq[NTO];
                if constexpr (TAB) {
                    tq[0] = tv.x;
                    tq[NTO > 1 ? 1 : 0] = NTO > 1 ? tv.y : tq[0];
                    tq[NTO > 2 ? 2 : 0] = NTO > 2 ? tv.z : tq[0];
                    tq[NTO > 3 ? 3 : 0] = NTO > 3 ? tv.w : tq[0];
                } else {
#pragma unroll
                    for (int q = 0; q < NTO; ++q) tq[q] = tix[q];
                }
                // every row's taps read first (one LDS round trip), then summed in tap order
                float tvq[RP][NTO];
#pragma unroll
                for (int b = 0; b < RP; ++b)
#pragma unroll
                    for (int q = 0; q < NTO; ++q) tvq[b][q] = s_T[b * TSZ + tq[q]];
#pragma unroll
                for (int b = 0; b < RP; ++b) {
                    float acc = 0.f;
#pragma unroll
                    for (int q = 0; q < NTO; ++q) acc += tvq[b][q];
                    lbp[b] = fminf(acc * lo_o, acc * hi_o);
                    mag[b] = fabsf(acc) * fmaxf(fabsf(lo_o), fabsf(hi_o));
                    const bool neg = acc < 0.f;
                    s_x[b * XS + t] = neg ? hi_o : lo_o;
                    if (b < nb) {
                        xc_o += neg ? 1 : 0;
                        if (a.xbits) a.xbits[(long)(cr0 + ri + b) * d0 + t] = neg ? 1 : 0;
                    }
                }
            }
        } else {
            for (int o = t; o < d0; o += MBT) {
                const int ci = o / HiWi, qq = o - ci * HiWi;
                const int Yq = qq / a.Wi;
                const int Yp = Yq + a.p, Xp = qq - Yq * a.Wi + a.p;
                float l, h;
                if (a.box_lds) {
                    l = s_lo[o];
                    h = s_hi[o];
                } else {
                    l = glo[o];
                    h = ghi[o];
                }
#pragma unroll
                for (int b = 0; b < RP; ++b) {
                    float acc = 0.f;
#pragma unroll
                    for (int ty = 0; ty < (KK ? (KK + SS - 1) / SS : 8); ++ty) {
                        const int ky = Yp % s + ty * s;
                        if (!KK && ky >= k) break;
                        const int y = (Yp - ky) / s;
                        if (ky >= k || y < 0 || y >= a.Ho) continue;
#pragma unroll
                        for (int tx = 0; tx < (KK ? (KK + SS - 1) / SS : 8); ++tx) {
                            const int kx = Xp % s + tx * s;
                            if (!KK && kx >= k) break;
                            const int x = (Xp - kx) / s;
                            if (kx >= k || x < 0 || x >= a.Wo) continue;
                            acc += s_T[b * TSZ + ((ci * k + ky) * k + kx) * HP + y * a.Wo + x];
                        }
                    }
                    lbp[b] += fminf(acc * l, acc * h);
                    mag[b] += fabsf(acc) * fmaxf(fabsf(l), fabsf(h));
                    const bool neg = acc < 0.f;
                    s_x[b * XS + o] = neg ? h : l;
                    if (b < nb) {
                        if (a.adjoint && neg) s_xc[o] += 1;
                        if (a.xbits) a.xbits[(long)(cr0 + ri + b) * d0 + o] = neg ? 1 : 0;
                    }
                }
            }
        }
        // the owned tile's adjoint gathers (written once in the prologue), read before the barrier
        int4 gv4;
        if constexpr (TAB) gv4 = s_tab[MBT + t];
        // block sums of the RP rows' bound terms (one barrier, which also publishes s_x)
        {
            float vals[3 * RP];
#pragma unroll
            for (int b = 0; b < RP; ++b) {
                vals[3 * b] = wave_sum(lbp[b]);
                vals[3 * b + 1] = wave_sum(mag[b]);
                vals[3 * b + 2] = wave_sum(cpt[b]);
            }
            if (lane == 0)
#pragma unroll
                for (int q = 0; q < 3 * RP; ++q) red[q][wave] = vals[q];
            lds_sync();
            // the last wavefront (no position tile for most shapes) finishes the sums: lane q
            // adds red[q] in a fixed order, lane b the bound of row b
            if (wave == MNW - 1) {
                float tot = 0.f;
                if (lane < 3 * RP) {
                    const float* rq = red[lane];
                    const float h0 = ((rq[0] + rq[1]) + (rq[2] + rq[3])) + ((rq[4] + rq[5]) + (rq[6] + rq[7]));
                    const float h1 = ((rq[8] + rq[9]) + (rq[10] + rq[11])) + ((rq[12] + rq[13]) + (rq[14] + rq[15]));
                    tot = h0 + h1;
                }
                const int b = lane;
                const int src = min(3 * b, 3 * RP - 3);
                const float t0 = __shfl(tot, src), t1 = __shfl(tot, src + 1), t2 = __shfl(tot, src + 2);
                if (b < nb) {
                    const int r = cr0 + ri + b;
                    const RowDesc rd = s_rd[ri + b];
                    float lb = (t0 + t2) - (t1 + fabsf(t2)) * a.margin;   // rounding margin of spec rows
                    if (!(lb == lb) || isinf(lb)) lb = -INFINITY;
                    const float old = s_old[ri + b];
                    if (a.mode == 0) {
                        const long e = (long)in.slot * a.ld_state + a.state_off_obj + rd.j;
                        if (rd.sign > 0)
                            a.lw[e] = fmaxf(old, lb);
                        else
                            a.uw[e] = fminf(old, isinf(lb) ? INFINITY : -lb);
                    } else {
                        a.lb_out[r] = lb;
                        if (a.mode == 1) {
                            const bool better = lb > old;
                            if (better) a.best[r] = lb;
                            a.improved[r] = better ? 1 : 0;
                        }
                    }
                }
            }
        }
        if (a.adjoint) {
            // ---- adjoint: ghat^T = W1 im2col(x*)^T + b1 on the owned tile, then the relaxation of
            // ReLU layer 0 and the alpha (and MNC g) sums of the owned neurons, rows in order
            f4 acc[RP];
#pragma unroll
            for (int b = 0; b < RP; ++b) acc[b] = f4{0.f, 0.f, 0.f, 0.f};
            if (mt < MT) {
                int gq[KSM];
                if constexpr (TAB) {
                    gq[0] = gv4.x;
                    gq[KSM > 1 ? 1 : 0] = KSM > 1 ? gv4.y : gq[0];
                    gq[KSM > 2 ? 2 : 0] = KSM > 2 ? gv4.z : gq[0];
                    gq[KSM > 3 ? 3 : 0] = KSM > 3 ? gv4.w : gq[0];
                } else {
#pragma unroll
                    for (int ks = 0; ks < KSM; ++ks) gq[ks] = gidx[ks];
                }
#pragma unroll
                for (int ks = 0; ks < KSM; ++ks) {
                    if (4 * ks >= ntap) break;
                    const int gi = gq[ks];
#pragma unroll
                    for (int b = 0; b < RP; ++b) {
                        const float xv = s_x[b * XS + gi];
                        acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aW[ks], xv, acc[b], 0, 0, 0);
                    }
                }
            }
            // O1: the four relaxations and the bias in one LDS round trip (otherwise each where
            // it is used: fewer live registers)
            float4 rxa[4], b1q;
            if constexpr (O1) {
#pragma unroll
                for (int v = 0; v < 4; ++v) rxa[v] = relax(v);
                b1q = s_b1[lk];
            }
            float gv[RP][4];
            if constexpr (!O1) b1q = s_b1[lk];
            const float b1g[4] = {b1q.x, b1q.y, b1q.z, b1q.w};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float4 rx = O1 ? rxa[v] : relax(v);
                float sg = 0.f;
#pragma unroll
                for (int b = 0; b < RP; ++b) {
                    // lane holds ghat[co = 4 lk + v][pos] without the bias
                    const float gh = acc[b][v] + b1g[v];
                    const float p = ap[b][v];
                    const bool neg = p < 0.f;
                    const float g = (neg ? rx.y : rx.x) * gh + (neg ? rx.z : 0.f);
                    if (b < nb) {
                        if (rx.z > 0.f && !neg) da[v] += p * gh;
                        if constexpr (O1) sg += g;
                        else if (a.gsum_out && pv) s_sg[(4 * lk + v) * HoWo + pos] += g;
                    }
                    gv[b][v] = g;
                }
                // O1: the rows' g in row order, one LDS update per neuron
                if (O1 && a.gsum_out && pv) s_sg[(4 * lk + v) * HoWo + pos] += sg;
            }
            if constexpr (PFL) mf_drain(); else vmem_drain();
            if (a.Gout && pv) {
#pragma unroll
                for (int b = 0; b < RP; ++b)
                    if (b < nb)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            float* growp = a.Gout + (long)(cr0 + ri + b) * d1;
                            growp[(4 * lk + v) * HoWo + pos] = gv[b][v];
                        }
            }
        } else {
            if constexpr (PFL) mf_drain(); else vmem_drain();
        }
        // next iteration: its T writes follow the barrier above (every col2im read is done) and
        // its x* writes follow its first barrier (every adjoint gather of this one is done)
    }
    if (!a.adjoint) return;
    lds_sync();   // s_sg and s_xc complete
    // partial sums of this chunk: alpha only where the neuron is unstable, the g sum only for
    // MNCs, and per input element the number of rows with x* = hi
    float* pt = a.part + (long)blockIdx.x * (2 * d1 + d0);
    if (pv)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = (4 * lk + v) * HoWo + pos;
            if (relax(v).z > 0.f) pt[j] = da[v];
            if (a.gsum_out) pt[d1 + j] = s_sg[j];
        }
    if constexpr (O1) {
        if (t < d0) pt[2 * d1 + t] = (float)xc_o;
    } else {
        for (int o = t; o < d0; o += MBT) pt[2 * d1 + o] = (float)s_xc[o];
    }
}

template <int TPW, int KK, int SS, int NTT, bool O1>
void launch_mf_o1(const BottomArgs& a, size_t lds, hipStream_t st) {
    if (a.src_mode == 0)
        hipLaunchKernelGGL((k_bottom_mf<TPW, KK, SS, NTT, false, O1>), dim3(a.n_chunk), dim3(MBT), lds, st, a);
    else
        hipLaunchKernelGGL((k_bottom_mf<TPW, KK, SS, NTT, true, O1>), dim3(a.n_chunk), dim3(MBT), lds, st, a);
}

template <int TPW, int KK, int SS, int NTT>
void launch_mf_src(const BottomArgs& a, size_t lds, hipStream_t st) {
    if (a.d0 <= MBT)
        launch_mf_o1<TPW, KK, SS, NTT, true>(a, lds, st);
    else
        launch_mf_o1<TPW, KK, SS, NTT, false>(a, lds, st);
}

template <int KK, int SS, int NTT>
void launch_mf_tpw(const BottomArgs& a, size_t lds, hipStream_t st) {
    launch_mf_src<1, KK, SS, NTT>(a, lds, st);
}

}  // namespace

// Compile-time shape (KK, SS) and tap tiles of the instantiation launch_bottom_mf picks.
static void mf_shape(int Ci, int k, int s, int& KK, int& SS, int& ntt) {
    ntt = Ci * k * k > 16 ? 2 : 1;
    KK = SS = 0;
    if (ntt == 1 && k == 4 && s == 2) KK = 4, SS = 2;
    if (ntt == 2 && k == 3 && s == 2) KK = 3, SS = 2;
}

// LDS of the MFMA bottom kernel without the box: relaxation, the rows' tap products and x*,
// x* counts, g sums (MNC), per-thread index tables (as the kernel lays them out)
static size_t mf_lds(int Ci, int k, int s, int Ho, int Wo, int d0, int d1, bool mnc) {
    int KK, SS, ntt;
    mf_shape(Ci, k, s, KK, SS, ntt);
    const size_t rp = mf_rows(KK, ntt);
    const bool tab = mf_tab(d0 <= MBT, KK, SS, ntt);
    const size_t hp = 16 * (size_t)((Ho * Wo + 15) / 16) + 1;   // padded tap stride of T
    return (4 * (size_t)d1 + rp * 16 * ntt * hp + rp * ((size_t)d0 + 1) + d0 + (mnc ? (size_t)d1 : 0) +
            (tab ? 4 + 2 * 4 * (size_t)MBT : 0)) *
           sizeof(float);
}

// Dynamic LDS the kernel may take next to its static arrays (with the LDS prefetch: its slots,
// 4 KB per row of an iteration, and under 2 KB of descriptors and sums) within the CU's 160 KB.
static size_t mf_dyn_limit(int Ci, int k, int s, int d0) {
    int KK, SS, ntt;
    mf_shape(Ci, k, s, KK, SS, ntt);
    if (!mf_pf_lds(false, d0 <= MBT)) return 150 * 1024;
    return 160 * 1024 - (size_t)MNW * mf_rows(KK, ntt) * 256 * sizeof(float) - 2048;
}

bool bottom_mf_supported(int Co, int Ci, int k, int s, int Ho, int Wo, int d0, int d1, bool mnc) {
    const int HoWo = Ho * Wo, ntap = Ci * k * k;
    const size_t lds = mf_lds(Ci, k, s, Ho, Wo, d0, d1, mnc);
    return Co == 16 && ntap <= 32 && (HoWo + 15) / 16 <= MNW && lds <= mf_dyn_limit(Ci, k, s, d0);
}

void launch_bottom_mf(const BottomArgs& a, hipStream_t st) {
    const int HoWo = a.Ho * a.Wo, ntap = a.Ci * a.k * a.k;
    MNB_CHECK(bottom_mf_supported(a.Co, a.Ci, a.k, a.s, a.Ho, a.Wo, a.d0, a.d1, a.gsum_out != nullptr) && a.d1 == 16 * HoWo,
              MNB_EDEVICE, "bottom kernel (MFMA): unsupported shape");
    const int ntt = ntap > 16 ? 2 : 1;
    size_t lds = mf_lds(a.Ci, a.k, a.s, a.Ho, a.Wo, a.d0, a.d1, a.gsum_out != nullptr);
    BottomArgs b = a;
    // with one input element per thread (d0 <= MBT) the box is held in registers instead
    b.box_lds = a.d0 > MBT && lds + 2 * (size_t)a.d0 * sizeof(float) <= mf_dyn_limit(a.Ci, a.k, a.s, a.d0);
    if (b.box_lds) lds += 2 * (size_t)a.d0 * sizeof(float);
    if (ntt == 1 && a.k == 4 && a.s == 2)
        launch_mf_tpw<4, 2, 1>(b, lds, st);
    else if (ntt == 2 && a.k == 3 && a.s == 2)
        launch_mf_tpw<3, 2, 2>(b, lds, st);
    else if (ntt == 1)
        launch_mf_tpw<0, 0, 1>(b, lds, st);
    else
        launch_mf_tpw<0, 0, 2>(b, lds, st);
    MNB_HIP(hipGetLastError());
}

}  // namespace mnb
