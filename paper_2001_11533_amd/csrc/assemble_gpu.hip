// P1 finite-element assembly on the GPU (paper, Section 2: [A]_ij =
// a(phi_j, phi_i), [M]_ij = (phi_j, phi_i)), bit-identical to the host
// assembler: one thread forms one row, visiting the row vertex's elements in
// ascending element index and adding each element's contributions with the
// shared element arithmetic (p1_element.hpp, no fused multiply-add), exactly
// the order in which the host adds them.
//
// Steps: vertex -> element lists (counts, exclusive scan, placement, then a
// per-vertex sort so each list is ascending whatever order the placement
// took); per row the sorted distinct neighbours by repeated wavefront-minimum
// search over the row vertex's elements (counts, scan, fill); then the values.
#include <climits>
#include <cstdint>
#include <mutex>

#include "common.hpp"
#include "p1_element.hpp"

#pragma clang fp contract(off)

namespace amg {
namespace {

constexpr int kAsmBlock = 256;

int blocks_for(long n) {
    long b = (n + kAsmBlock - 1) / kAsmBlock;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}

__global__ void k_ids_in_range(long n, const int32_t *ids, int32_t nv, int *bad) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        if (ids[i] < 0 || ids[i] >= nv) *bad = 1;
}

__global__ void k_vertex_count(long n, const int32_t *ids, int32_t *cnt) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        atomicAdd(&cnt[ids[i]], 1);
}

// out[0..n]: exclusive sums of in[0..n-1], out[n] the total, in three
// launches over chunks of kScanChunk entries: chunk sums (coalesced loads),
// their exclusive scan by one workgroup (which flags a total beyond int32),
// then each chunk scanned in its workgroup from its offset.
constexpr int kScanPer = 8, kScanChunk = kAsmBlock * kScanPer;

__device__ long long block_sum(long long v, long long *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int o = kAsmBlock / 2; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    const long long r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kAsmBlock) void k_scan_chunks(int32_t n, const int32_t *in, long long *csum) {
    __shared__ long long red[kAsmBlock];
    const long c0 = (long)blockIdx.x * kScanChunk;
    long long s = 0;
    for (int i = 0; i < kScanPer; ++i) {
        const long j = c0 + (long)i * kAsmBlock + threadIdx.x;
        if (j < n) s += in[j];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) csum[blockIdx.x] = s;
}

__global__ void k_scan_offsets(int nchunks, long long *csum, int32_t n, int32_t *out, int *over) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long long run = 0;
    for (int c = 0; c < nchunks; ++c) {
        const long long v = csum[c];
        csum[c] = run;
        run += v;
    }
    out[n] = run > INT_MAX ? INT_MAX : (int32_t)run;
    if (run > INT_MAX) *over = 1;
}

__global__ __launch_bounds__(kAsmBlock) void k_scan_write(int32_t n, const int32_t *in, const long long *coff,
                                                          int32_t *out) {
    __shared__ long long part[kAsmBlock];
    const int t = threadIdx.x;
    const long base = (long)blockIdx.x * kScanChunk + (long)t * kScanPer;  // this thread's entries
    int32_t v[kScanPer];
    long long s = 0;
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    part[t] = s;
    __syncthreads();
    if (t == 0) {  // exclusive scan of the thread sums, in order
        long long run = coff[blockIdx.x];
        for (int k = 0; k < kAsmBlock; ++k) {
            const long long x = part[k];
            part[k] = run;
            run += x;
        }
    }
    __syncthreads();
    long long run = part[t];
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < n) out[base + i] = run > INT_MAX ? INT_MAX : (int32_t)run;
        run += v[i];
    }
}

__global__ void k_vertex_place(int32_t ne, int nl, const int32_t *elems, const int32_t *vp, int32_t *fill,
                               int32_t *ve) {
    const long n = (long)ne * nl;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int32_t v = elems[i];
        ve[vp[v] + atomicAdd(&fill[v], 1)] = (int32_t)(i / nl);
    }
}

// each vertex's element list in ascending order (insertion sort: the lists
// are as long as the number of elements around a vertex)
__global__ void k_vertex_sort(int32_t nv, const int32_t *vp, int32_t *ve) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
        const int32_t p0 = vp[v], p1 = vp[v + 1];
        for (int32_t p = p0 + 1; p < p1; ++p) {
            const int32_t x = ve[p];
            int32_t q = p - 1;
            while (q >= p0 && ve[q] > x) {
                ve[q + 1] = ve[q];
                --q;
            }
            ve[q + 1] = x;
        }
    }
}

// Row lengths (count) or columns (fill) of the mesh graph, sorted and
// distinct: one wavefront per row.  The candidates are the vertices of the row
// vertex's elements (candidate c: vertex c % nl of its (c / nl)-th element);
// lane l holds candidates l and l + 64 in registers and reads any further ones
// from memory.  Each step takes the smallest candidate above the last one by a
// wavefront minimum (INT_MAX, never a vertex id, marks none).
template <bool FILL>
__global__ void k_row_pattern(int32_t nv, int nl, const int32_t *elems, const int32_t *vp, const int32_t *ve,
                              int32_t *cnt, const int32_t *rowptr, int32_t *col) {
    const int lane = threadIdx.x & 63;
    const long w0 = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6;
    const long nw = ((long)gridDim.x * blockDim.x) >> 6;
    for (long v = w0; v < nv; v += nw) {
        const int32_t p0 = vp[v];
        const int32_t nc = (vp[v + 1] - p0) * nl;
        auto cand = [&](int32_t c) { return elems[(long)ve[p0 + c / nl] * nl + c % nl]; };
        const int32_t c0 = lane < nc ? cand(lane) : INT_MAX;
        const int32_t c1 = lane + 64 < nc ? cand(lane + 64) : INT_MAX;
        const int32_t base = FILL ? rowptr[v] : 0;
        int32_t last = -1, m = 0;
        for (;;) {
            int32_t best = INT_MAX;
            if (c0 > last) best = c0;
            if (c1 > last && c1 < best) best = c1;
            for (int32_t c = lane + 128; c < nc; c += 64) {
                const int32_t k = cand(c);
                if (k > last && k < best) best = k;
            }
            for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
            if (best == INT_MAX) break;  // the same value in every lane: the loop ends for the wavefront
            if constexpr (FILL)
                if (lane == 0) col[base + m] = best;
            ++m;
            last = best;
        }
        if constexpr (!FILL)
            if (lane == 0) cnt[v] = m;
    }
}

// DIM is a template parameter so that the small coordinate and gradient arrays
// stay in registers (all their indices are compile-time after unrolling; the
// row's own gradient is picked by predication).
template <int DIM>
__global__ void k_row_values(int32_t nv, const double *coords, const int32_t *elems, const double *kappa,
                             const int32_t *vp, const int32_t *ve, const int32_t *rowptr, const int32_t *col,
                             double *valA, double *valM) {
    constexpr int NL = DIM + 1;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
        const int32_t r0 = rowptr[v], r1 = rowptr[v + 1];
        for (int32_t q = r0; q < r1; ++q) {
            valA[q] = 0.0;
            valM[q] = 0.0;
        }
        for (int32_t p = vp[v]; p < vp[v + 1]; ++p) {  // elements in ascending order
            const int32_t e = ve[p];
            const int32_t *ev = elems + (long)e * NL;
            int32_t vid[NL];
            double X[NL * DIM];
#pragma unroll
            for (int a = 0; a < NL; ++a) {
                vid[a] = ev[a];
#pragma unroll
                for (int r = 0; r < DIM; ++r) X[a * DIM + r] = coords[(long)vid[a] * DIM + r];
            }
            // the row of the element matrices that belongs to v, formed by the
            // same helpers (hence the same operations) as the host's full matrices
            double g[4][3];
            double meas;
            p1_grads(DIM, X, g, meas);
            const double w = kappa[e] * meas;
            int a = 0;  // v's place in the element (its first, as on the host)
#pragma unroll
            for (int b = NL - 1; b >= 0; --b)
                if (vid[b] == v) a = b;
            double ga[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) ga[r] = 0.0;
#pragma unroll
            for (int b = 0; b < NL; ++b)
                if (b == a) {
#pragma unroll
                    for (int r = 0; r < DIM; ++r) ga[r] = g[b][r];
                }
#pragma unroll
            for (int b = 0; b < NL; ++b) {
                const int32_t k = vid[b];
                int32_t lo = r0, hi = r1;  // first position with col >= k
                while (lo < hi) {
                    const int32_t mid = lo + (hi - lo) / 2;
                    if (col[mid] < k) lo = mid + 1;
                    else hi = mid;
                }
                valA[lo] = valA[lo] + p1_stiff_vec(DIM, ga, g[b], w);
                valM[lo] = valM[lo] + p1_mass(DIM, meas, a, b);
            }
        }
    }
}

#define ASM_HIP(x)                                                                   \
    do {                                                                             \
        const hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? AMG_ERR_OOM : AMG_ERR_HIP; \
    } while (0)

// fills n ints with v (used instead of a memset node, so the clears stay
// kernels of the caller's stream)
__global__ void k_fill(long n, int32_t *p, int32_t v) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

// The temporary arrays of one assembly, carved from one workspace: error
// flags, chunk sums of the scans, row counts, the vertex -> element lists
// (vp, ve) and the mesh graph's row pointers (rp).
struct AsmScratch {
    int *flags = nullptr;      // [2]: vertex id out of range, total beyond int32
    long long *csum = nullptr; // [chunks]
    int32_t *cnt = nullptr, *vp = nullptr, *ve = nullptr, *rp = nullptr;
};

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t scratch_bytes(int dim, int32_t nv, int32_t ne) {
    const size_t nid = (size_t)ne * (dim + 1), nv1 = (size_t)nv + 1;
    const size_t chunks = ((size_t)nv + kScanChunk - 1) / kScanChunk;
    return round256(2 * sizeof(int)) + round256(chunks * sizeof(long long)) + 3 * round256(nv1 * sizeof(int32_t)) +
           round256(nid * sizeof(int32_t));
}

AsmScratch carve(void *base, int dim, int32_t nv, int32_t ne) {
    const size_t nid = (size_t)ne * (dim + 1), nv1 = (size_t)nv + 1;
    const size_t chunks = ((size_t)nv + kScanChunk - 1) / kScanChunk;
    char *p = static_cast<char *>(base);
    AsmScratch a;
    auto take = [&](size_t b) {
        char *q = p;
        p += round256(b);
        return q;
    };
    a.flags = (int *)take(2 * sizeof(int));
    a.csum = (long long *)take(chunks * sizeof(long long));
    a.cnt = (int32_t *)take(nv1 * sizeof(int32_t));
    a.vp = (int32_t *)take(nv1 * sizeof(int32_t));
    a.ve = (int32_t *)take(nid * sizeof(int32_t));
    a.rp = (int32_t *)take(nv1 * sizeof(int32_t));
    return a;
}

// A workspace from the process-wide cache of device blocks (a block of a
// little more than the size asked for, or a new allocation), handed back to
// the cache, not freed, once the stream has run the work that uses it: so
// repeated assemblies call neither hipMalloc nor hipFree (which waits for the
// whole device).
struct PoolBlock {
    int dev = -1;
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t s = nullptr;
    int get(size_t b, hipStream_t st) {
        s = st;
        ASM_HIP(hipGetDevice(&dev));
        auto got = DevPool::get().take(dev, b);
        if (!got.first) {
            void *q = nullptr;
            hipError_t e = hipMalloc(&q, b);
            if (e != hipSuccess) {  // once more without the cached blocks of this device
                (void)hipGetLastError();
                DevPool::get().release(dev);
                e = hipMalloc(&q, b);
            }
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return e == hipErrorOutOfMemory ? AMG_ERR_OOM : AMG_ERR_HIP;
            }
            got = {q, b};
        }
        p = got.first;
        bytes = got.second;
        return AMG_OK;
    }
    ~PoolBlock() {
        if (!p) return;
        (void)hipStreamSynchronize(s);
        if (!DevPool::get().give(dev, p, bytes)) (void)hipFree(p);
    }
};

void scan(int32_t n, const int32_t *in, int32_t *out, long long *csum, int *over, hipStream_t s) {
    const int nchunks = (int)(((long)n + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_scan_chunks, dim3(nchunks), dim3(kAsmBlock), 0, s, n, in, csum);
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(64), 0, s, nchunks, csum, n, out, over);
    hipLaunchKernelGGL(k_scan_write, dim3(nchunks), dim3(kAsmBlock), 0, s, n, in, (const long long *)csum, out);
}

// vertex -> element lists (vp[nv+1], ve ascending per vertex) and the row
// lengths of the mesh graph with their scan (rp[nv+1]); *total gets rp[nv]
int mesh_lists(int dim, int32_t nv, int32_t ne, const int32_t *elems, hipStream_t s, const AsmScratch &w,
               int32_t *total) {
    const int nl = dim + 1;
    const long nid = (long)ne * nl;
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, 2L, (int32_t *)w.flags, 0);
    hipLaunchKernelGGL(k_fill, dim3(blocks_for((long)nv + 1)), dim3(kAsmBlock), 0, s, (long)nv + 1, w.cnt, 0);
    hipLaunchKernelGGL(k_ids_in_range, dim3(blocks_for(nid)), dim3(kAsmBlock), 0, s, nid, elems, nv, w.flags);
    int h[4] = {0, 0, 0, 0};  // host words of the two read-backs
    ASM_HIP(hipMemcpyAsync(h, w.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    ASM_HIP(hipStreamSynchronize(s));
    if (h[0]) return AMG_ERR_ARG;  // out-of-range vertex ids: nothing below indexes with them
    hipLaunchKernelGGL(k_vertex_count, dim3(blocks_for(nid)), dim3(kAsmBlock), 0, s, nid, elems, w.cnt);
    scan(nv, w.cnt, w.vp, w.csum, w.flags + 1, s);
    hipLaunchKernelGGL(k_fill, dim3(blocks_for((long)nv + 1)), dim3(kAsmBlock), 0, s, (long)nv + 1, w.cnt, 0);
    hipLaunchKernelGGL(k_vertex_place, dim3(blocks_for(nid)), dim3(kAsmBlock), 0, s, ne, nl, elems, w.vp, w.cnt,
                       w.ve);
    hipLaunchKernelGGL(k_vertex_sort, dim3(blocks_for(nv)), dim3(kAsmBlock), 0, s, nv, w.vp, w.ve);
    hipLaunchKernelGGL((k_row_pattern<false>), dim3(blocks_for(64L * nv)), dim3(kAsmBlock), 0, s, nv, nl, elems,
                       w.vp, w.ve, w.cnt, (const int32_t *)nullptr, (int32_t *)nullptr);
    scan(nv, w.cnt, w.rp, w.csum, w.flags + 1, s);
    ASM_HIP(hipGetLastError());
    ASM_HIP(hipMemcpyAsync(h + 2, w.rp + nv, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ASM_HIP(hipMemcpyAsync(h + 3, w.flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    ASM_HIP(hipStreamSynchronize(s));
    if (h[3]) return AMG_ERR_ARG;  // more than 2^31 - 1 entries
    *total = h[2];
    return AMG_OK;
}

// the pattern and values into the caller's arrays (nnz checked against the
// mesh graph first)
int assemble_into(int dim, int32_t nv, const double *coords, int32_t ne, const int32_t *elems, const double *kappa,
                  int32_t nnz, int32_t *rowptr, int32_t *col, double *valA, double *valM, hipStream_t s,
                  const AsmScratch &w) {
    int32_t tot = 0;
    if (int e = mesh_lists(dim, nv, ne, elems, s, w, &tot)) return e;
    if (tot != nnz) return AMG_ERR_ARG;  // the caller's arrays do not fit this pattern
    const int nl = dim + 1;
    ASM_HIP(hipMemcpyAsync(rowptr, w.rp, sizeof(int32_t) * ((size_t)nv + 1), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL((k_row_pattern<true>), dim3(blocks_for(64L * nv)), dim3(kAsmBlock), 0, s, nv, nl, elems,
                       (const int32_t *)w.vp, (const int32_t *)w.ve, (int32_t *)nullptr, rowptr, col);
    if (dim == 2)
        hipLaunchKernelGGL((k_row_values<2>), dim3(blocks_for(nv)), dim3(kAsmBlock), 0, s, nv, coords, elems, kappa,
                           (const int32_t *)w.vp, (const int32_t *)w.ve, rowptr, col, valA, valM);
    else
        hipLaunchKernelGGL((k_row_values<3>), dim3(blocks_for(nv)), dim3(kAsmBlock), 0, s, nv, coords, elems, kappa,
                           (const int32_t *)w.vp, (const int32_t *)w.ve, rowptr, col, valA, valM);
    ASM_HIP(hipGetLastError());
    ASM_HIP(hipStreamSynchronize(s));
    return AMG_OK;
}

// ---- the allocation-free variant ----
// Its workspace is this file-scope device array: every device that runs the
// call holds one copy until the process ends, and every call on a device
// reuses that device's copy (so calls that overlap on one device race).
constexpr size_t kNoAllocBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// The array's device address, looked up once per device with that device
// current; host code uses these addresses, never the array's name (which on
// the host is only a stand-in symbol).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void **out) {
    int dev = -1;
    ASM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return AMG_ERR_ARG;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        ASM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return AMG_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return AMG_OK;
}

bool valid_args(int dim, int32_t nv, int32_t ne, const int32_t *elems) {
    return (dim == 2 || dim == 3) && nv > 0 && ne > 0 && elems && (long)ne * (dim + 1) <= INT_MAX;
}

}  // namespace
}  // namespace amg

extern "C" int amg_p1_pattern_device(int dim, int32_t nv, int32_t ne, const int32_t *elems, int32_t *nnz,
                                     void *stream) {
    using namespace amg;
    if (!nnz || !valid_args(dim, nv, ne, elems)) return AMG_ERR_ARG;
    const hipStream_t s = (hipStream_t)stream;
    PoolBlock blk;
    if (int e = blk.get(scratch_bytes(dim, nv, ne), s)) return e;
    return mesh_lists(dim, nv, ne, elems, s, carve(blk.p, dim, nv, ne), nnz);
}

extern "C" int amg_p1_assemble_device(int dim, int32_t nv, const double *coords, int32_t ne, const int32_t *elems,
                                      const double *kappa, int32_t nnz, int32_t *rowptr, int32_t *col,
                                      double *valA, double *valM, void *stream) {
    using namespace amg;
    if (!coords || !kappa || !rowptr || !col || !valA || !valM || !valid_args(dim, nv, ne, elems))
        return AMG_ERR_ARG;
    const hipStream_t s = (hipStream_t)stream;
    PoolBlock blk;
    if (int e = blk.get(scratch_bytes(dim, nv, ne), s)) return e;
    return assemble_into(dim, nv, coords, ne, elems, kappa, nnz, rowptr, col, valA, valM, s,
                         carve(blk.p, dim, nv, ne));
}

extern "C" int amg_p1_assemble_device_noalloc(int dim, int32_t nv, const double *coords, int32_t ne,
                                              const int32_t *elems, const double *kappa, int32_t nnz,
                                              int32_t *rowptr, int32_t *col, double *valA, double *valM,
                                              void *stream) {
    using namespace amg;
    if (!coords || !kappa || !rowptr || !col || !valA || !valM || !valid_args(dim, nv, ne, elems))
        return AMG_ERR_ARG;
    if (scratch_bytes(dim, nv, ne) > kNoAllocBytes) return AMG_ERR_ARG;  // beyond the static workspace
    void *base = nullptr;
    if (int e = scratch_of_current_device(&base)) return e;
    return assemble_into(dim, nv, coords, ne, elems, kappa, nnz, rowptr, col, valA, valM, (hipStream_t)stream,
                         carve(base, dim, nv, ne));
}
