// Common definitions of the amghess library (gfx950): error handling, device
// allocations, CSR containers and launch geometry.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "amghess.h"

namespace amg {

struct Error {
    int code;
    std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw Error{code, msg}; }

#define AMG_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            ::amg::fail(e_ == hipErrorOutOfMemory ? AMG_ERR_OOM : AMG_ERR_HIP,             \
                        std::string(#call) + ": " + hipGetErrorString(e_));                \
    } while (0)

// Every device allocation of a context goes through one arena so that a
// failure anywhere in setup releases everything.
struct Arena {
    std::vector<void *> ptrs;
    size_t bytes = 0;
    template <class T> T *alloc(size_t n) {
        if (n == 0) n = 1;
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, n * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(AMG_ERR_OOM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
        }
        ptrs.push_back(p);
        bytes += n * sizeof(T);
        return static_cast<T *>(p);
    }
    void release(void *p) {
        for (auto &q : ptrs)
            if (q == p) {
                (void)hipFree(q);
                q = nullptr;
            }
    }
    void free_all() {
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
    }
};

// CSR matrix in device memory: int32 indices, FP64 values and an optional
// float32 copy of the values for the mixed-precision path.
struct DCsr {
    int n = 0, m = 0, nnz = 0;
    int *rp = nullptr;
    int *ci = nullptr;
    double *v = nullptr;
    float *v32 = nullptr;
};

constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts of 64)
constexpr int kMaxGrid = 16384;        // workgroups at most for kernels with reductions
constexpr int kMaxGridPlain = 1 << 20; // and for kernels without
constexpr int kFinBlock = 1024;        // threads of a finalize kernel
constexpr int kXcd = 8;          // XCDs of an MI355X

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Grid for a row-blocked kernel: a multiple of 8 so that the XCD-aware remap
// (see xcd_block) is a permutation.
inline int grid_rows(long rows, int rows_per_block, int maxg = kMaxGrid) {
    int g = ceil_div(rows, rows_per_block);
    if (g > maxg) g = maxg;
    if (g < 1) g = 1;
    return ceil_div(g, kXcd) * kXcd;
}

}  // namespace amg
