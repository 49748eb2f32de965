// Shared internal definitions of the MN-BaB MI355X engine (host + device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace mnb {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};
void set_error(int code, const std::string& msg);

#define MNB_HIP(expr)                                                                \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            throw ::mnb::Error{-3, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define MNB_CHECK(cond, code, msg)                     \
    do {                                               \
        if (!(cond)) throw ::mnb::Error{(code), (msg)}; \
    } while (0)

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
// Largest grid.y (and grid.z) of one launch; kernels with rows on grid.y are launched in slices.
constexpr int kMaxGridY = 65535;

// ---------------------------------------------------------------- device helpers
// v + the value of the lane `CTRL` selects (a DPP row shift or row broadcast), 0 where the
// source lane lies outside the row or the row is masked off.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_src(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, true));
}

// Sum over the 64 lanes of a wavefront, in a fixed order, returned to every lane.  Within each
// 16-lane row, row shifts by 1, 2, 4 and 8 leave the row total in the row's last lane; row
// broadcasts of lanes 15 and 31 then combine the four rows in lane 63, which is read back.
// Every lane of the wavefront must be active.
// Sums over each 16-lane row of the wavefront, valid in the row's last lane (15, 31, 47, 63).
__device__ __forceinline__ float row16_sum(float v) {
    v += dpp_src<0x111, 0xF>(v);   // row_shr:1
    v += dpp_src<0x112, 0xF>(v);   // row_shr:2
    v += dpp_src<0x114, 0xF>(v);   // row_shr:4
    v += dpp_src<0x118, 0xF>(v);   // row_shr:8
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_src<0x111, 0xF>(v);   // row_shr:1
    v += dpp_src<0x112, 0xF>(v);   // row_shr:2
    v += dpp_src<0x114, 0xF>(v);   // row_shr:4
    v += dpp_src<0x118, 0xF>(v);   // row_shr:8
    v += dpp_src<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_src<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// c_r plus the ncp partial constants of the ReLU folds (row r of cpart), summed by one
// wavefront: lane q adds the partials q, q + 64, ..., then the lanes are combined in a fixed
// order.  All loads are issued together; every lane returns the total.
__device__ __forceinline__ float row_constant(const float* c, const float* cpart, int ldcp, int ncp, long r) {
    float s = 0.f;
    for (int kq = (int)(threadIdx.x & 63); kq < ncp; kq += 64) s += cpart[r * ldcp + kq];
    return c[r] + wave_sum(s);
}

// Wait until every global load and store this thread issued has completed (vmcnt 0; the LDS
// and scalar counters are left alone).  The vector-memory counter covers loads and stores
// alike, so a row loop that loads one row ahead drains it where those loads have long
// arrived: nothing is then outstanding at the top of the next row, and no wait there also
// waits for the stores of the row before.
__device__ __forceinline__ void vmem_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Kernel variants forced by mnb_set_kernel_variants (bits MNB_VAR_* of mnbab.h).
int kernel_variants();

// ---------------------------------------------------------------- descriptors passed to kernels
// Per-row descriptor of a back-substitution pass: which subproblem (local index
// into the call's slot list), which parameter set, which instance (subproblem,
// set) and, for intermediate-bound rows, the neuron and sign.
struct RowDesc {
    int32_t b;      // local subproblem index
    int32_t inst;   // instance index (rows of one instance share a parameter set)
    int32_t j;      // objective neuron (intermediate rows) or spec row index
    int32_t sign;   // +1 lower-bound row, -1 upper-bound row, 0 spec row
};

// Instance = (local subproblem, parameter set) with a contiguous row range.
struct InstDesc {
    int32_t b;      // local subproblem index
    int32_t slot;   // global slot index
    int32_t set;    // parameter-set index
    int32_t r0, r1; // row range [r0, r1)
};

}  // namespace mnb
