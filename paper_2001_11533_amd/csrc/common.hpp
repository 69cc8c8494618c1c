// Common definitions of the amghess library (gfx950): error handling, device
// allocations, CSR containers and launch geometry.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <utility>
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

// Device blocks that ended contexts give back, kept per device for later
// contexts of the process (what a framework's caching allocator does): a
// context then starts and ends without hipMalloc / hipFree calls, each of
// which waits for the device.  A request takes the smallest cached block of
// its device that is at least as large and at most a third larger;
// amg_release_memory hands every cached block back to the driver.
struct DevPool {
    struct Blk {
        int dev;
        size_t bytes;
        void *p;
    };
    std::mutex m;
    std::vector<Blk> blks;
    size_t held = 0;
    static constexpr size_t kMaxHeld = size_t(32) << 30;
    // never destroyed: no hipFree may run after the runtime has shut down
    static DevPool &get() {
        static DevPool *pool = new DevPool();
        return *pool;
    }
    // a cached block (and its size) or {nullptr, 0}
    std::pair<void *, size_t> take(int dev, size_t bytes) {
        std::lock_guard<std::mutex> g(m);
        int best = -1;
        for (size_t i = 0; i < blks.size(); ++i)
            if (blks[i].dev == dev && blks[i].bytes >= bytes && blks[i].bytes <= bytes + bytes / 3 &&
                (best < 0 || blks[i].bytes < blks[best].bytes))
                best = (int)i;
        if (best < 0) return {nullptr, 0};
        const Blk b = blks[best];
        blks.erase(blks.begin() + best);
        held -= b.bytes;
        return {b.p, b.bytes};
    }
    // false: not kept (the cache is full), the caller frees it
    bool give(int dev, void *p, size_t bytes) {
        std::lock_guard<std::mutex> g(m);
        if (held + bytes > kMaxHeld) return false;
        blks.push_back({dev, bytes, p});
        held += bytes;
        return true;
    }
    // every cached block of device dev (all devices when dev < 0) to the driver
    void release(int dev) {
        std::vector<Blk> out;
        {
            std::lock_guard<std::mutex> g(m);
            std::vector<Blk> keep;
            for (const Blk &b : blks) (dev < 0 || b.dev == dev ? out : keep).push_back(b);
            blks.swap(keep);
            for (const Blk &b : out) held -= b.bytes;
        }
        for (const Blk &b : out) (void)hipFree(b.p);
    }
};

// Every device allocation of a context goes through one arena so that a
// failure anywhere in setup releases everything.  Requests up to a quarter of a
// chunk are carved from large chunks (few hipMalloc calls, and few hipFree
// calls when the context ends: each waits for the device); larger ones get
// their own allocation.  A released block is kept and handed out again to a
// later request of at most its size (and at least half of it): all work of a
// context runs in order on its one stream, so the kernels that used the block
// are ahead of any that reuse it.
struct Arena {
    struct Blk {
        void *p;
        size_t bytes;
        bool live;
    };
    std::vector<Blk> blks;                         // every block handed out
    std::vector<std::pair<void *, size_t>> chunks; // device allocations (cached or new) and sizes
    int dev = -1;                                  // device of the allocations
    char *cur = nullptr;
    size_t cur_left = 0, next_chunk = size_t(8) << 20;
    size_t bytes = 0;
    static constexpr size_t kMaxChunk = size_t(128) << 20;

    void *dev_malloc(size_t b) {
        if (dev < 0 && hipGetDevice(&dev) != hipSuccess) fail(AMG_ERR_HIP, "hipGetDevice failed");
        auto got = DevPool::get().take(dev, b);
        if (!got.first) {
            void *p = nullptr;
            hipError_t e = hipMalloc(&p, b);
            if (e != hipSuccess) {  // once more without the cache's blocks of this device
                (void)hipGetLastError();
                DevPool::get().release(dev);
                e = hipMalloc(&p, b);
            }
            if (e != hipSuccess) {
                (void)hipGetLastError();
                fail(AMG_ERR_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed");
            }
            got = {p, b};
        }
        chunks.push_back(got);
        bytes += got.second;
        return got.first;
    }
    template <class T> T *alloc(size_t n) {
        if (n == 0) n = 1;
        const size_t want = (n * sizeof(T) + 255) & ~(size_t)255;
        Blk *best = nullptr;
        for (auto &b : blks)
            if (!b.live && b.bytes >= want && b.bytes <= 2 * want && (!best || b.bytes < best->bytes)) best = &b;
        if (best) {
            best->live = true;
            return static_cast<T *>(best->p);
        }
        void *p;
        if (want > kMaxChunk / 4) {
            p = dev_malloc(want);
        } else {
            if (want > cur_left) {
                const size_t c = std::max(next_chunk, want);
                cur = static_cast<char *>(dev_malloc(c));
                cur_left = c;
                next_chunk = std::min(kMaxChunk, 2 * next_chunk);
            }
            p = cur;
            cur += want;
            cur_left -= want;
        }
        blks.push_back({p, want, true});
        return static_cast<T *>(p);
    }
    void release(void *p) {
        for (auto &b : blks)
            if (b.p == p) b.live = false;
    }
    // back to the process's cache (the context's streams have drained)
    void free_all() {
        for (auto &ch : chunks)
            if (!DevPool::get().give(dev, ch.first, ch.second)) (void)hipFree(ch.first);
        chunks.clear();
        blks.clear();
        cur = nullptr;
        cur_left = 0;
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
    // optional sliced-ELL copy (finest level): slices of 64 rows stored column
    // by column, entry k of row 64 s + l at sl_off[s] + 64 k + l; a column is
    // kept as a 16-bit offset from the slice's smallest column sl_base[s] (the
    // copy exists only when every slice spans fewer than 65536 columns), and the
    // rows of a slice are padded to its longest with (offset 0, value 0)
    int nsl = 0;
    bool sl_over8 = true;   // some slice is wider than 8 entries per row
    int *sl_off = nullptr;  // [nsl + 1]
    int *sl_base = nullptr; // [nsl]
    uint16_t *sl_cd = nullptr;
    double *sl_v = nullptr;
    float *sl_v32 = nullptr;
    // lanes-per-row choice set by the autotuner: log2 G for batch width
    // 2^k (k = 0..4) and values FP64 (0) / float32 (1); -1 = the default rule
    int8_t tuned_lg[5][2] = {{-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}};
};

constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts of 64)
constexpr int kMaxGrid = 16384;        // workgroups at most for kernels with reductions
constexpr int kMaxGridPlain = 1 << 20; // and for kernels without
// Reducing launches on NB columns: the partials of a finalize grow as grid x NB,
// so wide batches take fewer (fuller) workgroups.
template <int NB> constexpr int red_grid_max() { return NB <= 2 ? kMaxGrid : (2 * kMaxGrid) / NB; }
constexpr int kFinBlock = 1024;        // threads of a finalize kernel
constexpr int kXcd = 8;          // XCDs of an MI355X

__host__ __device__ inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Grid for a row-blocked kernel: a multiple of 8 so that the XCD-aware remap
// (see xcd_block) is a permutation.
inline int grid_rows(long rows, int rows_per_block, int maxg = kMaxGrid) {
    int g = ceil_div(rows, rows_per_block);
    if (g > maxg) g = maxg;
    if (g < 1) g = 1;
    return ceil_div(g, kXcd) * kXcd;
}

}  // namespace amg
