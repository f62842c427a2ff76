// Shared definitions of the tile-low-rank Matern likelihood library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>

#include "../../include/tlrmle.h"

namespace tlr {

// Returns TLR_E_HIP from the enclosing function when a HIP call fails.
#define TLR_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t err__ = (expr);                                                      \
        if (err__ != hipSuccess) {                                                      \
            std::fprintf(stderr, "tlrmle: %s failed: %s (%s:%d)\n", #expr,              \
                         hipGetErrorString(err__), __FILE__, __LINE__);                 \
            return TLR_E_HIP;                                                           \
        }                                                                               \
    } while (0)

#define TLR_TRY(expr)                          \
    do {                                       \
        tlr_status st__ = (expr);              \
        if (st__ != TLR_OK) return st__;       \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device-side parameter and status block at the start of every workspace.
struct DevParams {
    double sigma2, beta, nu, tol;
    double nu_coef;          // sigma2 / (Gamma(nu) 2^(nu-1)) for the general-nu kernel
    int32_t nu_kind;         // 0 general, 1 nu=1/2, 2 nu=3/2, 3 nu=5/2
    int32_t status;          // TLR_OK or first failure code
    int32_t fail_i, fail_j;  // tile of first failure
    int32_t dense_ok;        // over-rank tiles are kept dense by the host: not a failure
    int32_t pad1;
    // truncation floor relative to the operator's norm when the low-rank
    // factors are stored in float32 (0: float64 factors, plain tol)
    double floor_rel;
};

// First failure wins: record code and tile unless a failure is already stored.
__device__ inline void set_status(DevParams *p, int code, int i, int j) {
    if (atomicCAS(&p->status, 0, code) == 0) {
        p->fail_i = i;
        p->fail_j = j;
    }
}

// A rank above the cap: a failure unless the plan keeps such tiles dense
// (the host then sees the numerical rank in the tile's status words).
__device__ inline void rank_overflow(DevParams *p, int i, int j) {
    if (!p->dense_ok) set_status(p, TLR_RANK_OVERFLOW, i, j);
}

}  // namespace tlr
