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

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ float wave_sum(float v) {
    // Fixed-order butterfly over the 64 lanes of a wavefront.
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
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
