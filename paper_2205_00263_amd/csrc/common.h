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
