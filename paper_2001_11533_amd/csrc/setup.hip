// Smoothed-aggregation setup on the GPU (gfx950).
//
// The paper (Section 3.1) builds its Hessian preconditioner from the
// prolongators and Galerkin matrices of an AMG hierarchy built for the
// forward problem, and fixes ideas on smoothed aggregation.  This file builds
// that hierarchy with the following rules (every floating-point value is
// formed by IEEE operations in a fixed order, with no fused multiply-add, so
// the result is reproducible bit for bit):
//   strength   (i,k), k != i, both non-Dirichlet, strong iff
//              a_ik*a_ik >= t*(a_ii*a_kk), t = theta_j^2, theta_j = theta0 2^-j
//   roots      distance-2 maximal independent set of the strong graph taken
//              greedily by decreasing priority (splitmix64(seed^(j<<40)^i), i),
//              computed by fixed-priority rounds (a node joins when its key is
//              the largest among undecided nodes within two hops)
//   aggregates root r -> coarse id #{roots < r}; a node next to a root joins the
//              root with the largest |a_ir| (ties: smaller r); the rest join the
//              aggregate of the neighbour of the previous phase with the
//              largest |a_ik| (ties: smaller k)
//   prolongator S = (I - omega D^{-1} A) P_tent, P_tent[i, agg(i)] = 1,
//              omega = (4/3)/max_i(sum_k |a_ik| / a_ii), sums in column order
//   Galerkin   eqs. coarsestiffness/coarsemass with P_j = S_j: T = A S summed
//              over ascending k, then S^T T over ascending i, lower triangle
//              copied from the upper one
#include <algorithm>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <initializer_list>
#include <mutex>
#include <thread>

#include "ctx.hpp"

#pragma clang fp contract(off)

namespace amg {

namespace {

constexpr int kHS = 2048;        // LDS hash slots per wavefront in the sparse product
constexpr int kMaxRowOut = 1024; // output columns per row at most

// Atomics from many wavefronts on one word are serialised (roughly 10 ns per
// wavefront instruction), so reductions into a single word combine within the
// wavefront first, and a maximum is only sent when it raises the stored one
// (the stored value only grows, so a stale read never skips a needed update).
// Orders the LDS and memory accesses of one wavefront around a point every
// lane of it reaches: release fence, wavefront barrier, acquire fence.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_max(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ int wave_sum(int v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
template <class T> __device__ __forceinline__ void raise_max(T *dst, T v) {
    if (v > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, v);
}

// Per-row kernels with kRowLanes lanes per row: a row's entries are taken
// kRowLanes at a time, one per lane; ballots keep the row's order where it
// matters (compactions) and sequential sums fold the lanes' values in order.
constexpr int kRowLanes = 16;
__device__ __forceinline__ int row_lane() { return threadIdx.x % kRowLanes; }
__device__ __forceinline__ int row_first() { return (int)((blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes); }
__device__ __forceinline__ int row_stride() { return (int)(gridDim.x * blockDim.x / kRowLanes); }
// this lane's group's bits of a wavefront ballot (every lane of the group takes part)
__device__ __forceinline__ unsigned group_bits(bool pred) {
    const unsigned long long b = __ballot(pred);
    return (unsigned)((b >> ((threadIdx.x % 64) / kRowLanes * kRowLanes)) & 0xFFFFull);
}
__device__ __forceinline__ unsigned lanes_below() { return (1u << row_lane()) - 1u; }

__global__ void k_check_sym(int n, const int *rp, const int *ci, const double *v, int *bad) {
    const int gl = row_lane();
    for (int i = row_first(); i < n; i += row_stride()) {
        const int e = rp[i + 1];
        for (int p = rp[i] + gl; p < e; p += kRowLanes) {
            const int k = ci[p];
            if (k < 0 || k >= n) {
                atomicAdd(bad, 1);
                continue;
            }
            int lo = rp[k], hi = rp[k + 1] - 1, found = -1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = ci[mid];
                if (cm == i) {
                    found = mid;
                    break;
                }
                if (cm < i) lo = mid + 1;
                else hi = mid - 1;
            }
            if (found < 0 || __double_as_longlong(v[found]) != __double_as_longlong(v[p]))
                atomicAdd(bad, 1);
            if (p > rp[i] && ci[p - 1] >= k) atomicAdd(bad + 1, 1);  // unsorted / duplicate
        }
    }
}

__global__ void k_diag(int n, const int *rp, const int *ci, const double *v, const uint8_t *mask,
                       double *d, int *bad) {
    const int gl = row_lane();
    for (int i = row_first(); i < n; i += row_stride()) {
        double di = 0.0;
        const int e = rp[i + 1];
        for (int p0 = rp[i]; p0 < e; p0 += kRowLanes) {  // the last stored diagonal entry, as a serial loop
            const int p = p0 + gl;
            const bool hit = p < e && ci[p] == i;
            const double x = hit ? v[p] : 0.0;
            const unsigned b = group_bits(hit);
            const double y = __shfl(x, b ? 31 - __clz(b) : 0, kRowLanes);
            if (b) di = y;
        }
        if (gl == 0) {
            d[i] = di;
            if (!(di > 0.0) && !(mask && mask[i])) atomicAdd(bad, 1);
        }
    }
}

// A_0 = D A D + (I - D) (D = diag(1 - mask), mask null: D = I): Dirichlet rows
// and columns leave the pattern, the Dirichlet diagonal is one, and A's stored
// zeros are dropped (an off-diagonal entry stays only when it is nonzero, the
// diagonal always); counts, then the fill.
__device__ __forceinline__ bool a0_keep(int i, int k, double v, const uint8_t *mask) {
    return !(mask && mask[k]) && (v != 0.0 || k == i);
}

__global__ void k_a0_count(int n, const int *rp, const int *ci, const double *v, const uint8_t *mask, int *cnt) {
    const int gl = row_lane();
    for (int i = row_first(); i < n; i += row_stride()) {
        if (mask && mask[i]) {
            if (gl == 0) cnt[i] = 1;
            continue;
        }
        int c = 0;
        const int e = rp[i + 1];
        for (int p0 = rp[i]; p0 < e; p0 += kRowLanes) {
            const int p = p0 + gl;
            c += __popc(group_bits(p < e && a0_keep(i, ci[p], v[p], mask)));
        }
        if (gl == 0) cnt[i] = c;
    }
}

__global__ void k_a0_fill(int n, const int *rp, const int *ci, const double *v, const uint8_t *mask,
                          const int *rp0, int *ci0, double *v0) {
    const int gl = row_lane();
    for (int i = row_first(); i < n; i += row_stride()) {
        int o = rp0[i];
        if (mask && mask[i]) {
            if (gl == 0) {
                ci0[o] = i;
                v0[o] = 1.0;
            }
            continue;
        }
        const int e = rp[i + 1];
        for (int p0 = rp[i]; p0 < e; p0 += kRowLanes) {
            const int p = p0 + gl;
            const bool keep = p < e && a0_keep(i, ci[p], v[p], mask);
            const unsigned b = group_bits(keep);
            if (keep) {
                const int r = __popc(b & lanes_below());
                ci0[o + r] = ci[p];
                v0[o + r] = v[p];
            }
            o += __popc(b);
        }
    }
}

// exclusive scan in two passes over blocks of kScanPer counts: the block sums,
// then per block its offset (the sum of the block sums before it) and its part
// of the scan by wavefront shuffles; the last block writes out[n] and *total
constexpr int kScanPer = 1024;
constexpr int kScanPT = kScanPer / kBlock;  // counts per thread
__global__ __launch_bounds__(kBlock) void k_scan_blocks(int n, const int *in, int *bsum) {
    __shared__ int ws[kBlock / 64];
    const int t = threadIdx.x, i0 = blockIdx.x * kScanPer + t * kScanPT;
    int acc = 0;
#pragma unroll
    for (int q = 0; q < kScanPT; ++q) {
        const int v = in[min(i0 + q, n - 1)];  // n >= 1 here
        acc += i0 + q < n ? v : 0;
    }
    acc = wave_sum(acc);
    if ((t & 63) == 0) ws[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
        int b = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) b += ws[w];
        bsum[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_final(int n, int nb, const int *in, const int *bsum, int *out,
                                                       int *total) {
    __shared__ int ws[kBlock / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int o = 0;
    for (int b = t; b < (int)blockIdx.x; b += kBlock) o += bsum[b];
    o = wave_sum(o);
    if (lane == 0) ws[w] = o;
    __syncthreads();
    int off = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) off += ws[q];
    __syncthreads();
    const int i0 = blockIdx.x * kScanPer + t * kScanPT;
    int v[kScanPT], tsum = 0;
#pragma unroll
    for (int q = 0; q < kScanPT; ++q) {
        const int x = n > 0 ? in[min(i0 + q, n - 1)] : 0;
        v[q] = i0 + q < n ? x : 0;
        tsum += v[q];
    }
    int inc = tsum;  // inclusive scan of the thread sums over the wavefront
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    int run = off + inc - tsum;
    for (int q = 0; q < w; ++q) run += ws[q];
#pragma unroll
    for (int q = 0; q < kScanPT; ++q) {
        if (i0 + q < n) out[i0 + q] = run;
        run += v[q];
    }
    if (blockIdx.x == nb - 1 && t == kBlock - 1) {
        out[n] = run;
        *total = run;
    }
}

__global__ void k_l1(int n, const int *rp, const double *v, double *dl1inv, double *dl1) {
    const int gl = row_lane();
    for (int i = row_first(); i < n; i += row_stride()) {
        double s = 0.0;
        const int e = rp[i + 1];
        for (int p0 = rp[i]; p0 < e; p0 += kRowLanes) {
            const int p = p0 + gl;
            const double x = p < e ? fabs(v[p]) : 0.0;
            const int cn = min(kRowLanes, e - p0);
            for (int j = 0; j < cn; ++j) s = s + __shfl(x, j, kRowLanes);  // in the row's order
        }
        if (gl == 0) {
            dl1[i] = s;
            dl1inv[i] = 1.0 / s;
        }
    }
}

__global__ void k_inv(int n, const double *d, double *dinv) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dinv[i] = 1.0 / d[i];
}

__global__ void k_strength(int n, const int *rp, const int *ci, const double *v, const double *d,
                           const uint8_t *mask, double t, uint8_t *flag, int *cnt) {
    const int gl = row_lane();
    for (int i = row_first(); i < n; i += row_stride()) {
        int c = 0;
        const bool mi = mask && mask[i];
        const double di = d[i];
        const int e = rp[i + 1];
        for (int p0 = rp[i]; p0 < e; p0 += kRowLanes) {
            const int p = p0 + gl;
            bool s = false;
            if (p < e) {
                const int k = ci[p];
                if (k != i && !mi && !(mask && mask[k])) {
                    const double a = v[p];
                    const double lhs = a * a;
                    const double dd = di * d[k];
                    const double rhs = t * dd;
                    s = lhs >= rhs;
                }
                flag[p] = s;
            }
            c += __popc(group_bits(s));
        }
        if (gl == 0) cnt[i] = c;
    }
}

__global__ void k_strong_fill(int n, const int *rp, const int *ci, const double *v, const uint8_t *flag,
                              const int *srp, int *sci, double *sabs) {
    const int gl = row_lane();
    for (int i = row_first(); i < n; i += row_stride()) {
        int o = srp[i];
        const int e = rp[i + 1];
        for (int p0 = rp[i]; p0 < e; p0 += kRowLanes) {
            const int p = p0 + gl;
            const bool f = p < e && flag[p];
            const unsigned b = group_bits(f);
            if (f) {
                const int r = __popc(b & lanes_below());
                sci[o + r] = ci[p];
                sabs[o + r] = fabs(v[p]);
            }
            o += __popc(b);
        }
    }
}

// SplitMix64 output function (Steele, Lea and Flood, 2014): add the golden
// gamma, two xor-shift-multiply rounds, final xor-shift.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_hash(int n, uint64_t base, uint64_t *h) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        h[i] = splitmix64(base ^ (uint64_t)i);
}

enum : int8_t { UNDEC = 0, ROOT = 1, OUT = 2 };

__device__ __forceinline__ bool prio_gt(const uint64_t *h, int a, int b) {
    // (h[a], a) > (h[b], b); b < 0 means "none"
    if (a < 0) return false;
    if (b < 0) return true;
    const uint64_t ha = h[a], hb = h[b];
    return ha > hb || (ha == hb && a > b);
}

__global__ void k_mis_init(int n, const uint8_t *mask, int8_t *st) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        st[i] = (mask && mask[i]) ? OUT : UNDEC;
}

// Each round's kernels take the undecided count its predecessor left (null in
// the first round) and return at once when it is zero, so that rounds can be
// issued in batches ahead of the one read that ends the loop.
__device__ __forceinline__ bool mis_done(const int *prev) { return prev && *prev == 0; }

__global__ void k_mis_m1(int n, const int *srp, const int *sci, const uint64_t *h, const int8_t *st,
                         int *m1, const int *prev) {
    if (mis_done(prev)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int best = st[i] == UNDEC ? i : -1;
        for (int p = srp[i]; p < srp[i + 1]; ++p) {
            const int k = sci[p];
            if (st[k] == UNDEC && prio_gt(h, k, best)) best = k;
        }
        m1[i] = best;
    }
}

__global__ void k_mis_m2(int n, const int *srp, const int *sci, const uint64_t *h, const int *m1,
                         int8_t *st, const int *prev) {
    if (mis_done(prev)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (st[i] != UNDEC) continue;
        int best = m1[i];
        for (int p = srp[i]; p < srp[i + 1]; ++p) {
            const int k = m1[sci[p]];
            if (prio_gt(h, k, best)) best = k;
        }
        if (best == i) st[i] = ROOT;
    }
}

__global__ void k_mis_r1(int n, const int *srp, const int *sci, const int8_t *st, uint8_t *r1,
                         const int *prev) {
    if (mis_done(prev)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint8_t any = st[i] == ROOT;
        for (int p = srp[i]; p < srp[i + 1] && !any; ++p) any = st[sci[p]] == ROOT;
        r1[i] = any;
    }
}

__global__ void k_mis_r2(int n, const int *srp, const int *sci, const uint8_t *r1, int8_t *st, int *undec,
                         const int *prev) {
    if (mis_done(prev)) return;
    int left = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (st[i] != UNDEC) continue;
        bool any = r1[i];
        for (int p = srp[i]; p < srp[i + 1] && !any; ++p) any = r1[sci[p]];
        if (any) st[i] = OUT;
        else ++left;
    }
    // the rounds need only whether nodes are left: one add per workgroup, and
    // none once the counter is nonzero (a relaxed load instead of a contended
    // atomic)
    __shared__ int wl[kBlock / 64];
    left = wave_sum(left);
    if (threadIdx.x % 64 == 0) wl[threadIdx.x / 64] = left;
    __syncthreads();
    if (threadIdx.x == 0) {
        int b = 0;
        for (int w = 0; w < (int)blockDim.x / 64; ++w) b += wl[w];
        if (b && __hip_atomic_load(undec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) atomicAdd(undec, b);
    }
}

__global__ void k_root_flags(int n, const int8_t *st, uint8_t *root, int *cnt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        root[i] = st[i] == ROOT;
        cnt[i] = st[i] == ROOT;
    }
}

// phase 2: roots get their coarse id, nodes next to a root join the strongest root
__global__ void k_phase2(int n, const int *srp, const int *sci, const double *sabs, const uint8_t *root,
                         const int *cid, const uint8_t *mask, int *agg, uint8_t *p2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        p2[i] = 0;
        if (mask && mask[i]) {
            agg[i] = -1;
            continue;
        }
        if (root[i]) {
            agg[i] = cid[i];
            continue;
        }
        int bk = -1;
        double ba = 0.0;
        for (int p = srp[i]; p < srp[i + 1]; ++p) {
            const int k = sci[p];
            if (!root[k]) continue;
            const double a = sabs[p];
            if (bk < 0 || a > ba) {  // ascending k: ties keep the smaller k
                bk = k;
                ba = a;
            }
        }
        if (bk >= 0) {
            agg[i] = cid[bk];
            p2[i] = 1;
        } else {
            agg[i] = -2;
        }
    }
}

__global__ void k_phase3(int n, const int *srp, const int *sci, const double *sabs, const uint8_t *p2,
                         int *agg, int *unassigned) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (agg[i] != -2) continue;
        int bk = -1;
        double ba = 0.0;
        for (int p = srp[i]; p < srp[i + 1]; ++p) {
            const int k = sci[p];
            if (!p2[k]) continue;
            const double a = sabs[p];
            if (bk < 0 || a > ba) {
                bk = k;
                ba = a;
            }
        }
        if (bk >= 0) agg[i] = agg[bk];
        else atomicAdd(unassigned, 1);
    }
}

__global__ void k_rho(int n, const double *dl1, const double *d, const uint8_t *mask,
                      unsigned long long *maxbits) {
    // r > 0: the order of the bit patterns is the order of the values
    unsigned long long m = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (mask && mask[i]) continue;
        const double r = dl1[i] / d[i];
        m = max(m, (unsigned long long)__double_as_longlong(r));
    }
    for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, off));
    if (threadIdx.x % 64 == 0 && m) raise_max(maxbits, m);
}

// tentative prolongator: one unit entry per non-Dirichlet row
__global__ void k_ptent_count(int n, const int *agg, int *cnt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        cnt[i] = agg[i] >= 0 ? 1 : 0;
}

__global__ void k_ptent_fill(int n, const int *agg, const int *rp, int *ci, double *v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (agg[i] >= 0) {
            ci[rp[i]] = agg[i];
            v[rp[i]] = 1.0;
        }
}

// S[i,J] = [agg(i)=J] - (omega * s_iJ) / a_ii, s_iJ = (A P_tent)[i,J]
// omega = (4/3) / rho with rho the bit pattern k_rho left in *rhobits
__global__ void k_smooth(int n, const int *rp, const int *ci, double *v, const int *agg, const double *d,
                         const unsigned long long *rhobits) {
    const double omega = (4.0 / 3.0) / __longlong_as_double((long long)*rhobits);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const double t = omega * v[p];
            const double w = t / d[i];
            const double delta = ci[p] == agg[i] ? 1.0 : 0.0;
            v[p] = delta - w;
        }
    }
}

// transpose: counts, unordered placement, per-row insertion sort by row index
__global__ void k_t_count(int n, const int *rp, const int *ci, int *cnt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int p = rp[i]; p < rp[i + 1]; ++p) atomicAdd(&cnt[ci[p]], 1);
}

__global__ void k_t_place(int n, const int *rp, const int *ci, const double *v, const int *trp, int *fill,
                          int *tci, double *tv) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int J = ci[p];
            const int o = trp[J] + atomicAdd(&fill[J], 1);
            tci[o] = i;
            tv[o] = v[p];
        }
}

// Ordered transpose of a matrix with at most kTbCols columns, no atomics on
// global memory and no sort: blocks of kTbRows source rows count their
// entries per column in LDS (hist, column-major: column J, block b at
// J nb + b); an exclusive scan of hist gives every (column, block) its first
// position in the transpose; each block then places its entries in row order,
// so every row of the transpose comes out sorted by source row.
constexpr int kTbRows = 64, kTbCols = 8192, kTbChunk = 2048;
__global__ __launch_bounds__(kBlock) void k_tb_hist(int n, int nc, int nb, const int *rp, const int *ci,
                                                    int *hist) {
    __shared__ int lc[kTbCols];
    for (int J = threadIdx.x; J < nc; J += kBlock) lc[J] = 0;
    __syncthreads();
    static_assert(kTbRows * 4 == kBlock, "four lanes per row");
    const int i = blockIdx.x * kTbRows + threadIdx.x / 4;
    if (i < n)
        for (int p = rp[i] + threadIdx.x % 4; p < rp[i + 1]; p += 4) atomicAdd(&lc[ci[p]], 1);
    __syncthreads();
    for (int J = threadIdx.x; J < nc; J += kBlock) hist[(size_t)J * nb + blockIdx.x] = lc[J];
}

// pos: the scan of hist (pos[nc nb] = the total); block 0 also writes the
// transpose's row pointers trp[J] = pos[J nb].  Per chunk of the block's
// entries: columns staged in LDS, one wavefront hands out the positions row
// by row (the entries of a row have distinct columns, so its lanes never share
// a counter), then all threads write the entries.
__global__ __launch_bounds__(kBlock) void k_tb_place(int n, int nc, int nb, const int *rp, const int *ci,
                                                     const double *v, const int *pos, int *trp, int *tci,
                                                     double *tv) {
    __shared__ int lc[kTbCols];
    __shared__ int rps[kTbRows + 1];
    __shared__ int cj[kTbChunk], op[kTbChunk];
    const int t = threadIdx.x;
    for (int J = t; J < nc; J += kBlock) lc[J] = pos[(size_t)J * nb + blockIdx.x];
    if (blockIdx.x == 0)
        for (int J = t; J <= nc; J += kBlock) trp[J] = pos[(size_t)J * nb];
    const int r0 = blockIdx.x * kTbRows, nr = min(n, r0 + kTbRows) - r0;
    for (int q = t; q <= nr; q += kBlock) rps[q] = rp[r0 + q];
    __syncthreads();
    const int e0 = rps[0], e1 = rps[nr];
    for (int c0 = e0; c0 < e1; c0 += kTbChunk) {
        const int c1 = min(e1, c0 + kTbChunk);
        for (int p = c0 + t; p < c1; p += kBlock) cj[p - c0] = ci[p];
        __syncthreads();
        if (t < 64) {
            for (int r = 0; r < nr; ++r) {
                const int a = max(rps[r], c0), z = min(rps[r + 1], c1);
                for (int p0 = a; p0 < z; p0 += 64) {
                    const int p = p0 + t;
                    if (p < z) {
                        const int J = cj[p - c0];
                        const int o = lc[J];
                        lc[J] = o + 1;
                        op[p - c0] = o;
                    }
                    wave_sync();
                }
            }
        }
        __syncthreads();
        for (int p = c0 + t; p < c1; p += kBlock) {
            int lo = 0, hi = nr;  // the row of entry p: rps[lo] <= p < rps[lo + 1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) / 2;
                if (rps[mid] <= p) lo = mid;
                else hi = mid;
            }
            const int o = op[p - c0];
            tci[o] = r0 + lo;
            tv[o] = v[p];
        }
        __syncthreads();
    }
}

// rows of the transpose: rank sort by column index, one wavefront per row
// (the keys of a row are distinct row indices of the source matrix)
constexpr int kSortLds = 1024;  // keys of a row staged in LDS (longer rows read them from memory)
__global__ __launch_bounds__(kBlock) void k_row_sort(int m, const int *rp, const int *ci_in, const double *v_in,
                                                     int *ci_out, double *v_out) {
    __shared__ int keys[kBlock / 64][kSortLds];
    __shared__ int pos[kBlock / 64][kSortLds];
    const int lane = threadIdx.x % 64, wl = threadIdx.x / 64;
    const int w = (blockIdx.x * kBlock + threadIdx.x) / 64;
    const int nw = gridDim.x * kBlock / 64;
    for (int r = w; r < m; r += nw) {
        const int s = rp[r], e = rp[r + 1], len = e - s;
        if (len > 64 && len <= kSortLds) {
            // bitonic sort of (key, position) by the wavefront, padded with
            // INT_MAX keys to a power of two; the keys of a row are distinct
            int P = 128;
            while (P < len) P <<= 1;
            int *kk = keys[wl], *pp = pos[wl];
            for (int a = lane; a < P; a += 64) {
                kk[a] = a < len ? ci_in[s + a] : INT_MAX;
                pp[a] = a;
            }
            wave_sync();
            for (int k = 2; k <= P; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = lane; i < P; i += 64) {
                        const int ij = i ^ j;
                        if (ij > i) {
                            const int a = kk[i], b = kk[ij];
                            if ((a > b) == ((i & k) == 0)) {
                                kk[i] = b;
                                kk[ij] = a;
                                const int t = pp[i];
                                pp[i] = pp[ij];
                                pp[ij] = t;
                            }
                        }
                    }
                    wave_sync();
                }
            for (int a = lane; a < len; a += 64) {
                ci_out[s + a] = kk[a];
                v_out[s + a] = v_in[s + pp[a]];
            }
            wave_sync();
        } else if (len <= kSortLds) {
            for (int a = lane; a < len; a += 64) keys[wl][a] = ci_in[s + a];
            wave_sync();
            for (int a = lane; a < len; a += 64) {
                const int key = keys[wl][a];
                int rank = 0;
                for (int b = 0; b < len; ++b) rank += keys[wl][b] < key;
                ci_out[s + rank] = key;
                v_out[s + rank] = v_in[s + a];
            }
            wave_sync();
        } else {
            for (int a = s + lane; a < e; a += 64) {
                const int key = ci_in[a];
                int rank = 0;
                for (int b = s; b < e; ++b) rank += ci_in[b] < key;
                ci_out[s + rank] = key;
                v_out[s + rank] = v_in[a];
            }
        }
    }
}

// ---- sparse product C = A B, one wavefront per row of A, LDS hash of the
// output columns; values summed over the stored A[i,k] in ascending k ----

// steps of the numeric passes whose loads are issued together
constexpr int kPre = 8;

template <int HS> __device__ __forceinline__ void hs_insert(int *tab, int key, int *ucount, int *ovf) {
    unsigned h = ((unsigned)key * 2654435761u) & (HS - 1);
    for (int probe = 0; probe < HS; ++probe) {
        const int old = atomicCAS(&tab[h], -1, key);
        if (old == -1) {
            atomicAdd(ucount, 1);
            return;
        }
        if (old == key) return;
        h = (h + 1) & (HS - 1);
    }
    atomicOr(ovf, 1);
}

template <int HS> __device__ __forceinline__ int hs_find(const int *tab, int key) {
    unsigned h = ((unsigned)key * 2654435761u) & (HS - 1);
    for (int probe = 0; probe < HS; ++probe) {
        const int v = tab[h];
        if (v == key) return (int)h;
        if (v == -1) return -1;
        h = (h + 1) & (HS - 1);
    }
    return -1;
}

// Insert the columns of B[qb:qe) into the hash, loading them 8 at a time
// before the inserts so that their latencies overlap.  The loads are
// unconditional (past qe: the row's last entry again, then discarded), since
// guarded loads compile to one wait each.
template <int HS>
__device__ __forceinline__ void hs_insert_row(int *tab, const int *bci, int qb, int qe, int *ucount, int *ovf) {
    for (int q0 = qb; q0 < qe; q0 += 8) {
        int key[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = bci[min(q0 + i, qe - 1)];
            key[i] = q0 + i < qe ? k : -1;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (key[i] >= 0) hs_insert<HS>(tab, key[i], ucount, ovf);
    }
}

// Rank of key among the u distinct keys of ls (the number smaller than it).
// ls holds at least 8 INT_MAX sentinels after its u keys and is 16-byte
// aligned, so it is read in whole 16-byte vectors, several in flight.
__device__ __forceinline__ int rank_in(const int *ls, int u, int key) {
    int rank = 0;
#pragma unroll 2
    for (int f = 0; f < u; f += 8) {
        const int4 x0 = *reinterpret_cast<const int4 *>(ls + f);
        const int4 x1 = *reinterpret_cast<const int4 *>(ls + f + 4);
        rank += (x0.x < key) + (x0.y < key) + (x0.z < key) + (x0.w < key) + (x1.x < key) + (x1.y < key) +
                (x1.z < key) + (x1.w < key);
    }
    return rank;
}

// Symbolic pass, W wavefronts per row of A sharing one LDS hash of HS slots:
// output columns per row; maxes[0] and maxes[1] receive the largest output row
// and the longest row of B that is referenced.  With HS < kHS (first tier) a
// row whose outputs do not fit (or nearly fill) half the table gets cnt = -1 and maxes[2] = 1;
// the second tier (recount, HS = kHS) then counts only those rows.
template <int HS>
__device__ __forceinline__ void hs_insert_row_capped(int *tab, const int *bci, int qb, int qe, int *ucount,
                                                     int *full) {
    for (int q0 = qb; q0 < qe; q0 += 8) {
        int key[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {  // unconditional loads, as in hs_insert_row
            const int k = bci[min(q0 + i, qe - 1)];
            key[i] = q0 + i < qe ? k : -1;
        }
        // over the tier's capacity (checked per batch of 8): stop filling
        if (__hip_atomic_load(ucount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= HS / 2 - 8) {
            *full = 1;
            return;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (key[i] >= 0) hs_insert<HS>(tab, key[i], ucount, full);
    }
}

template <int W, int HS>
__global__ __launch_bounds__(64 * W) void k_spgemm_count(int n, const int *arp, const int *aci, const int *brp,
                                                         const int *bci, int *cnt, int *ovf, int *maxes,
                                                         int recount) {
    constexpr int NT = 64 * W;
    __shared__ int tab[HS];
    __shared__ int uc, full;
    __shared__ int red[2][W];
    const int t = threadIdx.x;
    int umax = 0, bmax = 0;
    for (int row = blockIdx.x; row < n; row += gridDim.x) {
        if (recount && cnt[row] >= 0) continue;  // counted by the first tier (uniform per workgroup)
        for (int s = t; s < HS; s += NT) tab[s] = -1;
        if (t == 0) {
            uc = 0;
            full = 0;
        }
        __syncthreads();
        for (int p = arp[row] + t; p < arp[row + 1]; p += NT) {
            const int k = aci[p];
            const int qb = brp[k], qe = brp[k + 1];
            bmax = max(bmax, qe - qb);
            if (HS < kHS) hs_insert_row_capped<HS>(tab, bci, qb, qe, &uc, &full);
            else hs_insert_row<HS>(tab, bci, qb, qe, &uc, ovf);
        }
        __syncthreads();
        if (t == 0) {
            if (HS < kHS && (full || uc > HS / 2)) {
                cnt[row] = -1;
                maxes[2] = 1;
            } else {
                cnt[row] = uc;
                umax = max(umax, uc);
                if (uc > kMaxRowOut) atomicOr(ovf, 1);
            }
        }
        __syncthreads();
    }
    for (int off = 32; off > 0; off >>= 1) {
        umax = max(umax, __shfl_xor(umax, off));
        bmax = max(bmax, __shfl_xor(bmax, off));
    }
    if (t % 64 == 0) {
        red[0][t / 64] = umax;
        red[1][t / 64] = bmax;
    }
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < W; ++w) {
            umax = max(umax, red[0][w]);
            bmax = max(bmax, red[1][w]);
        }
        raise_max(&maxes[0], umax);
        raise_max(&maxes[1], bmax);
    }
}

// Numeric pass, W wavefronts per row of A with an LDS hash of HS slots
// (HS / 2 >= the row's output count): rebuild the row's output columns, give
// each its rank in ascending order (its output position), then accumulate the
// products in LDS over the stored A[i,k] in ascending k.  The entries of the
// A row and the extents of the rows of B they select are staged in LDS.  The
// NT = 64 W threads form G groups of NT / G; one step hands G consecutive k
// to the groups (every row of B is at most NT / G long when G > 1), the
// groups then add their products one group after another with a barrier in
// between, and the loads of the next step are issued before those additions.
// For one k the products go to distinct outputs (the columns of row k of B
// are distinct), so every output entry receives its products strictly in
// ascending k: the rounded sums of a sequential loop.
template <int HS, int W>
__global__ __launch_bounds__(64 * W) void k_spgemm_fill(int n, int G, const int *arp, const int *aci,
                                                        const double *av, const int *brp, const int *bci,
                                                        const double *bv, const int *crp, int *cci, double *cv,
                                                        int *ovf) {
    constexpr int NT = 64 * W;
    __shared__ int tab[HS];
    __shared__ int pos[HS];
    __shared__ __align__(16) int lst[HS / 2 + 8];
    __shared__ double acc[HS / 2];
    __shared__ int sqb[NT], sqe[NT];
    __shared__ double sa[NT];
    __shared__ int uc, uc2;
    const int t = threadIdx.x;
    const int gs = NT / G, grp = t / gs, gl = t % gs;
    for (int row = blockIdx.x; row < n; row += gridDim.x) {
        for (int s = t; s < HS; s += NT) tab[s] = -1;
        if (t == 0) {
            uc = 0;
            uc2 = 0;
        }
        __syncthreads();
        const int a0 = arp[row], a1 = arp[row + 1];
        for (int p = a0 + t; p < a1; p += NT) {
            const int k = aci[p];
            hs_insert_row<HS>(tab, bci, brp[k], brp[k + 1], &uc, ovf);
        }
        __syncthreads();
        const int u = uc;
        if (u > HS / 2) {  // the host sized HS from the symbolic pass: cannot happen
            if (t == 0) atomicOr(ovf, 2);
            __syncthreads();
            continue;
        }
        for (int s = t; s < HS; s += NT) {
            const int key = tab[s];
            if (key >= 0) lst[atomicAdd(&uc2, 1)] = key;
        }
        if (t < 8) lst[u + t] = INT_MAX;  // sentinels for rank_in
        __syncthreads();
        const int cs = crp[row];
        for (int s = t; s < HS; s += NT) {
            const int key = tab[s];
            if (key < 0) continue;
            const int rank = rank_in(lst, u, key);
            pos[s] = rank;
            cci[cs + rank] = key;
            acc[rank] = 0.0;
        }
        for (int p0 = a0; p0 < a1; p0 += NT) {
            const int cnt = min(NT, a1 - p0);
            __syncthreads();  // ranks and zeroed sums done / previous chunk's staging no longer read
            if (t < cnt) {
                const int k = aci[p0 + t];
                sa[t] = av[p0 + t];
                sqb[t] = brp[k];
                sqe[t] = brp[k + 1];
            }
            __syncthreads();
            // kPre steps' loads at a time, unconditional (an empty slot reads a
            // valid entry and discards it; the product has entries)
            for (int eb = 0; eb < cnt; eb += kPre * G) {
                int pkey[kPre];
                double pval[kPre];
#pragma unroll
                for (int d = 0; d < kPre; ++d) {
                    const int e = min(eb + d * G + grp, cnt - 1);
                    const int qb = sqb[e], qe = eb + d * G + grp < cnt ? sqe[e] : qb;
                    const int q = max(min(qb + gl, qe - 1), 0);
                    const int kk = bci[q];
                    pval[d] = bv[q];
                    pkey[d] = qb + gl < qe ? kk : -1;
                }
#pragma unroll
            for (int d = 0; d < kPre; ++d) {
                const int e0 = eb + d * G;
                if (e0 >= cnt) break;
                const int e = e0 + grp;
                const int key = pkey[d];
                const double val = pval[d];
                int r = -1;
                double prod = 0.0;
                if (key >= 0) {
                    const int slot = hs_find<HS>(tab, key);
                    if (slot < 0) {  // cannot happen: every key was inserted above
                        atomicOr(ovf, 2);
                    } else {
                        r = pos[slot];
                        prod = sa[e] * val;
                    }
                }
                for (int g = 0; g < G; ++g) {
                    if (grp == g) {
                        if (r >= 0) acc[r] = acc[r] + prod;
                        if (G == 1 && e < cnt) {  // rows of B longer than NT: the rest of row k
                            const double a = sa[e];
                            for (int q = sqb[e] + NT + gl; q < sqe[e]; q += NT) {
                                const int slot = hs_find<HS>(tab, bci[q]);
                                if (slot < 0) {
                                    atomicOr(ovf, 2);
                                    continue;
                                }
                                const int r2 = pos[slot];
                                const double prod2 = a * bv[q];
                                acc[r2] = acc[r2] + prod2;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            }
        }
        __syncthreads();
        for (int e = t; e < u; e += NT) cv[cs + e] = acc[e];
        __syncthreads();
    }
}

// The same two passes for many short rows: a workgroup of kBlock threads
// holds kBlock / LPR groups of LPR lanes, each group on its own row with its
// own LDS hash of HS slots, so that many rows (and their chains of dependent
// loads) are in flight per CU.  A group's lanes lie in one wavefront, whose LDS
// accesses take effect in program order: the phases of a row are separated by
// wavefront syncs, not workgroup barriers, and the groups run independently.
//
// Symbolic pass: a row whose outputs do not fit (or nearly fill) HS / 2 gets cnt = -1 and
// maxes[2] = 1, and is counted again by k_spgemm_count with kHS slots.
template <int LPR, int HS>
__global__ __launch_bounds__(kBlock) void k_spgemm_count_sub(int n, const int *arp, const int *aci, const int *brp,
                                                             const int *bci, int *cnt, int *maxes) {
    constexpr int NG = kBlock / LPR;
    __shared__ int tab[NG][HS];
    __shared__ int uc[NG], full[NG];
    const int g = threadIdx.x / LPR, gl = threadIdx.x % LPR;
    int *tb = tab[g];
    int umax = 0, bmax = 0;
    for (int row = blockIdx.x * NG + g; row < n; row += gridDim.x * NG) {
        for (int s = gl; s < HS; s += LPR) tb[s] = -1;
        if (gl == 0) {
            uc[g] = 0;
            full[g] = 0;
        }
        wave_sync();
        const int a1 = arp[row + 1];
        for (int p = arp[row] + gl; p < a1; p += LPR) {
            const int k = aci[p];
            const int qb = brp[k], qe = brp[k + 1];
            bmax = max(bmax, qe - qb);
            hs_insert_row_capped<HS>(tb, bci, qb, qe, &uc[g], &full[g]);
        }
        wave_sync();
        if (gl == 0) {
            const int u = uc[g];
            if (full[g] || u > HS / 2) {
                cnt[row] = -1;
                maxes[2] = 1;  // a plain store: every writer stores 1
            } else {
                cnt[row] = u;
                umax = max(umax, u);
            }
        }
        wave_sync();
    }
    __shared__ int red[2][kBlock / 64];
    umax = wave_max(umax);
    bmax = wave_max(bmax);
    if (threadIdx.x % 64 == 0) {
        red[0][threadIdx.x / 64] = umax;
        red[1][threadIdx.x / 64] = bmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            umax = max(umax, red[0][w]);
            bmax = max(bmax, red[1][w]);
        }
        raise_max(&maxes[0], umax);
        raise_max(&maxes[1], bmax);
    }
}

// Numeric pass (HS / 2 >= every output count): the group inserts and ranks the
// row's columns as k_spgemm_fill does, then walks the stored A[i,k] in
// ascending k, LPR entries of the A row loaded at a time (one per lane) and
// handed out by shuffles.  A step gives GS = LPR / BL consecutive k to GS
// subgroups of BL lanes, one lane per entry of the row of B (a longer row
// takes further rounds); the loads of kPre steps are issued together, then
// those steps run, the subgroups of a step adding their products one after
// another.  For one k the products go to distinct outputs, so every output
// entry receives its products strictly in ascending k: the rounded sums of a
// sequential loop.  (B has at least one entry: the host launches no numeric
// pass for an empty product, so clamped indices are valid.)
template <int LPR, int HS, int BL>
__global__ __launch_bounds__(kBlock) void k_spgemm_fill_sub(int n, const int *arp, const int *aci,
                                                            const double *av, const int *brp, const int *bci,
                                                            const double *bv, const int *crp, int *cci, double *cv,
                                                            int *ovf) {
    constexpr int NG = kBlock / LPR, GS = LPR / BL;
    // fewer steps in flight for 16-lane groups (short rows of A, more groups per CU)
    constexpr int KP = LPR >= 32 ? kPre : kPre / 2;
    __shared__ int tab[NG][HS];
    __shared__ int pos[NG][HS];
    __shared__ __align__(16) int lst[NG][HS / 2 + 8];
    __shared__ double acc[NG][HS / 2];
    __shared__ int uc[NG], uc2[NG];
    const int g = threadIdx.x / LPR, gl = threadIdx.x % LPR, sg = gl / BL, sl = gl % BL;
    int *tb = tab[g], *ps = pos[g], *ls = lst[g];
    double *ac = acc[g];
    for (int row = blockIdx.x * NG + g; row < n; row += gridDim.x * NG) {
        for (int s = gl; s < HS; s += LPR) tb[s] = -1;
        if (gl == 0) {
            uc[g] = 0;
            uc2[g] = 0;
        }
        wave_sync();
        const int a0 = arp[row], a1 = arp[row + 1];
        for (int p = a0 + gl; p < a1; p += LPR) {
            const int k = aci[p];
            hs_insert_row<HS>(tb, bci, brp[k], brp[k + 1], &uc[g], ovf);
        }
        wave_sync();
        const int u = uc[g];
        if (u > HS / 2) {  // the host sized HS from the symbolic pass: cannot happen
            if (gl == 0) atomicOr(ovf, 2);
            wave_sync();
            continue;
        }
        for (int s = gl; s < HS; s += LPR) {
            const int key = tb[s];
            if (key >= 0) ls[atomicAdd(&uc2[g], 1)] = key;
        }
        if (gl < 8) ls[u + gl] = INT_MAX;  // sentinels for rank_in
        wave_sync();
        const int cs = crp[row];
        for (int s = gl; s < HS; s += LPR) {
            const int key = tb[s];
            if (key < 0) continue;
            const int rank = rank_in(ls, u, key);
            ps[s] = rank;
            cci[cs + rank] = key;
            ac[rank] = 0.0;
        }
        wave_sync();
        for (int c0 = a0; c0 < a1; c0 += LPR) {
            const int cn = min(LPR, a1 - c0);
            int mb = 0, me = 0;
            double ma = 0.0;
            if (gl < cn) {
                const int k = aci[c0 + gl];
                ma = av[c0 + gl];
                mb = brp[k];
                me = brp[k + 1];
            }
            const int nst = (cn + GS - 1) / GS;
            // step e takes entry e * GS + sg of the chunk (every lane of the
            // group takes part in the shuffles); KP steps' loads at a time,
            // unconditional (an empty slot reads a valid entry and discards it)
            for (int e0 = 0; e0 < nst; e0 += KP) {
                int pkey[KP], pqb[KP], pqe[KP];
                double pval[KP], pa[KP];
#pragma unroll
                for (int d = 0; d < KP; ++d) {
                    const int src = (e0 + d) * GS + sg;
                    const int qb = __shfl(mb, src, LPR);
                    int qe = __shfl(me, src, LPR);
                    pa[d] = __shfl(ma, src, LPR);
                    if (src >= cn) qe = qb;
                    const int q = max(min(qb + sl, qe - 1), 0);
                    const int kk = bci[q];
                    pval[d] = bv[q];
                    pkey[d] = qb + sl < qe ? kk : -1;
                    pqb[d] = qb;
                    pqe[d] = qe;
                }
#pragma unroll
            for (int d = 0; d < KP; ++d) {
                if (e0 + d >= nst) break;
                const int key = pkey[d], cb = pqb[d], ce = pqe[d];
                const double val = pval[d], ca = pa[d];
                int r = -1;
                double prod = 0.0;
                if (key >= 0) {
                    const int slot = hs_find<HS>(tb, key);
                    if (slot < 0) {  // cannot happen: every key was inserted above
                        atomicOr(ovf, 2);
                    } else {
                        r = ps[slot];
                        prod = ca * val;
                    }
                }
                for (int t2 = 0; t2 < GS; ++t2) {
                    if (sg == t2) {
                        if (r >= 0) ac[r] = ac[r] + prod;
                        for (int q = cb + BL + sl; q < ce; q += BL) {  // rows of B longer than BL
                            const int slot = hs_find<HS>(tb, bci[q]);
                            if (slot < 0) {
                                atomicOr(ovf, 2);
                                continue;
                            }
                            const int r2 = ps[slot];
                            const double prod2 = ca * bv[q];
                            ac[r2] = ac[r2] + prod2;
                        }
                    }
                    wave_sync();
                }
            }
            }
        }
        for (int e = gl; e < u; e += LPR) cv[cs + e] = ac[e];
        wave_sync();
    }
}

// The two passes when B has at most DC columns (the products from level 1
// down): one wavefront per row of A with a dense LDS accumulator and marker
// over B's columns instead of a hash, so a step is a plain indexed update.
// Symbolic: mark the columns reached (idempotent byte stores), count them.
template <int DC>
__global__ __launch_bounds__(64) void k_spgemm_count_dense(int n, const int *arp, const int *aci, const int *brp,
                                                           const int *bci, int *cnt, int *maxes) {
    __shared__ __align__(16) uint8_t mk[DC];
    const int lane = threadIdx.x;
    int umax = 0, bmax = 0;
    for (int row = blockIdx.x; row < n; row += gridDim.x) {
        for (int j = lane * 4; j < DC; j += 256) *reinterpret_cast<uint32_t *>(mk + j) = 0u;
        wave_sync();
        const int a1 = arp[row + 1];
        for (int p = arp[row] + lane; p < a1; p += 64) {
            const int k = aci[p];
            const int qb = brp[k], qe = brp[k + 1];
            bmax = max(bmax, qe - qb);
            for (int q0 = qb; q0 < qe; q0 += 8) {
                int key[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {  // unconditional loads, as in hs_insert_row
                    const int kk = bci[min(q0 + i, qe - 1)];
                    key[i] = q0 + i < qe ? kk : -1;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (key[i] >= 0) mk[key[i]] = 1;
            }
        }
        wave_sync();
        int c = 0;
        for (int j = lane * 4; j < DC; j += 256) c += __popc(*reinterpret_cast<const uint32_t *>(mk + j));
        c = wave_sum(c);
        if (lane == 0) cnt[row] = c;
        umax = max(umax, c);
        wave_sync();
    }
    umax = wave_max(umax);
    bmax = wave_max(bmax);
    if (lane == 0) {
        raise_max(&maxes[0], umax);
        raise_max(&maxes[1], bmax);
    }
}

// Numeric: the stored A[i,k] in ascending k, kPre steps' loads at a time; a
// step adds a[i,k] b[k,j] into acc[j] for the entries of row k of B, one per
// lane of the row's NW wavefronts (a row of B longer than 64 NW in further
// rounds of the same step).  The columns of one step are distinct, and the
// steps are ordered (a single wavefront's LDS accesses take effect in program
// order; several wavefronts wait at a barrier after each step), so acc[j]
// receives its products in ascending k from 0.0: the rounded sums of a
// sequential loop.  The row is written in ascending column order, as the hash
// passes write it.
template <int DC, int NW>
__global__ __launch_bounds__(64 * NW) void k_spgemm_fill_dense(int n, int m, const int *arp, const int *aci,
                                                               const double *av, const int *brp, const int *bci,
                                                               const double *bv, const int *crp, int *cci,
                                                               double *cv) {
    constexpr int NT = 64 * NW;
    __shared__ double acc[DC];
    __shared__ uint8_t mk[DC];
    __shared__ int sq[2][NT];
    __shared__ double sa[NT];
    const int t = threadIdx.x, lane = t & 63;
    auto sync = [&]() {
        if constexpr (NW == 1) wave_sync();
        else __syncthreads();
    };
    for (int row = blockIdx.x; row < n; row += gridDim.x) {
        for (int j = t; j < m; j += NT) {
            acc[j] = 0.0;
            mk[j] = 0;
        }
        const int a0 = arp[row], a1 = arp[row + 1];
        for (int c0 = a0; c0 < a1; c0 += NT) {
            const int cn = min(NT, a1 - c0);
            sync();  // zeroed sums / the previous chunk's staging no longer read
            {
                const int pc = c0 + min(t, cn - 1);  // threads past the chunk repeat its last entry (unused)
                const int k = aci[pc];
                sa[t] = av[pc];
                sq[0][t] = brp[k];
                sq[1][t] = brp[k + 1];
            }
            sync();
            for (int e0 = 0; e0 < cn; e0 += kPre) {
                int pkey[kPre];
                double pval[kPre];
#pragma unroll
                for (int d = 0; d < kPre; ++d) {
                    const int e = min(e0 + d, cn - 1);
                    const int qb = sq[0][e], qe = e0 + d < cn ? sq[1][e] : qb;
                    const int q = max(min(qb + t, qe - 1), 0);
                    const int kk = bci[q];
                    pval[d] = bv[q];
                    pkey[d] = qb + t < qe ? kk : -1;
                }
#pragma unroll
                for (int d = 0; d < kPre; ++d) {
                    const int e = e0 + d;
                    if (e >= cn) break;
                    const double a = sa[e];
                    const int key = pkey[d];
                    if (key >= 0) {
                        const double prod = a * pval[d];
                        acc[key] = acc[key] + prod;
                        mk[key] = 1;
                    }
                    for (int q = sq[0][e] + NT + t; q < sq[1][e]; q += NT) {  // rows of B longer than NT
                        const int j = bci[q];
                        const double prod = a * bv[q];
                        acc[j] = acc[j] + prod;
                        mk[j] = 1;
                    }
                    sync();
                }
            }
        }
        sync();
        if (t < 64) {  // the first wavefront writes the row
            const int cs = crp[row];
            int base = 0;
            for (int j0 = 0; j0 < m; j0 += 64) {
                const int j = j0 + lane;
                const bool on = j < m && mk[j];
                const unsigned long long bal = __ballot(on);
                if (on) {
                    const int p = base + __popcll(bal & ((1ull << lane) - 1));
                    cci[cs + p] = j;
                    cv[cs + p] = acc[j];
                }
                base += __popcll(bal);
            }
        }
        sync();
    }
}

// out[p] = S[i, ci[p]] over row i of T (zero where S has no entry), both rows
// sorted; a row of S with an entry outside T's row sets *bad
__global__ void k_align(int n, const int *trp, const int *tci, const int *srp, const int *sci, const double *sv,
                        double *out, int *bad) {
    const int gl = row_lane();
    for (int i = row_first(); i < n; i += row_stride()) {
        const int qb = srp[i], qe = srp[i + 1];
        const int e = trp[i + 1];
        int hit = 0;  // entries of S's row found in T's
        for (int p0 = trp[i]; p0 < e; p0 += kRowLanes) {
            const int p = p0 + gl;
            bool h = false;
            if (p < e) {
                const int k = tci[p];
                int lo = qb, hi = qe - 1, found = -1;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1;
                    const int cm = sci[mid];
                    if (cm == k) {
                        found = mid;
                        break;
                    }
                    if (cm < k) lo = mid + 1;
                    else hi = mid - 1;
                }
                h = found >= 0;
                out[p] = h ? sv[found] : 0.0;
            }
            hit += __popc(group_bits(h));
        }
        if (gl == 0 && hit != qe - qb) atomicOr(bad, 1);
    }
}

// lower triangle := upper triangle (symbolically symmetric pattern)
// one wavefront per row, lanes over the row's entries left of the diagonal
__global__ __launch_bounds__(kBlock) void k_mirror(int n, const int *rp, const int *ci, double *v, int *bad) {
    const int lane = threadIdx.x % 64;
    const int w = (blockIdx.x * kBlock + threadIdx.x) / 64;
    const int nw = gridDim.x * kBlock / 64;
    for (int i = w; i < n; i += nw) {
        for (int p = rp[i] + lane; p < rp[i + 1]; p += 64) {
            const int k = ci[p];
            if (k >= i) break;
            int lo = rp[k], hi = rp[k + 1] - 1, found = -1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = ci[mid];
                if (cm == i) {
                    found = mid;
                    break;
                }
                if (cm < i) lo = mid + 1;
                else hi = mid - 1;
            }
            if (found < 0) atomicAdd(bad, 1);
            else v[p] = v[found];
        }
    }
}

__global__ void k_to_f32(long n, const double *a, float *b) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

__global__ void k_to_u16(long n, const int *a, uint16_t *b) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        b[i] = (uint16_t)a[i];
}

// ---- dense kernels (coarsest level) ----
__global__ __launch_bounds__(kBlock) void k_densify(int n, const int *rp, const int *ci, const double *v,
                                                    const uint8_t *rmask, const uint8_t *cmask, double *D) {
    const int lane = threadIdx.x % 64;
    const int w = (blockIdx.x * kBlock + threadIdx.x) / 64;
    const int nw = gridDim.x * kBlock / 64;
    for (int i = w; i < n; i += nw) {
        const bool rk = !(rmask && rmask[i]);
        for (int p = rp[i] + lane; p < rp[i + 1]; p += 64) {
            const int k = ci[p];
            const bool ck = !(cmask && cmask[k]);
            D[(size_t)i * n + k] = (rk && ck) ? v[p] : 0.0;
        }
    }
}

// Dense inverses (tiles of kTB): every dense kernel below works on a batch of
// matrices of one order n stored back to back (matrix blockIdx.z at
// D + blockIdx.z * n * n).  They are compared with the oracle within a
// tolerance, not bit for bit: fused multiply-add is allowed there.
#pragma clang fp contract(fast)
constexpr int kTB = 32;

__device__ __forceinline__ double *bat(double *D, int n) { return D + (size_t)blockIdx.z * n * n; }
__device__ __forceinline__ const double *bat(const double *D, int n) { return D + (size_t)blockIdx.z * n * n; }

// kTB x kTB tiles in LDS; 256 threads each own a 2x2 block of a product tile.
typedef double Tile[kTB][kTB + 1];

typedef double v4d __attribute__((ext_vector_type(4)));

// The thread's 2x2 block (rows ra, ra+1; columns cb, cb+1) of the product
// P Q of two tiles, on the FP64 matrix cores: wavefront w forms the 16 x 16
// block (w / 2, w % 2) in kTB / 4 steps of v_mfma_f64_16x16x4f64 (lane l gives
// P[16 bi + l % 16][4 s + l / 16] and Q[4 s + l / 16][16 bj + l % 16], and holds
// Z[16 bi + l / 16 + 4 r][16 bj + l % 16] in its r-th result), the blocks pass
// through the tile Z to the threads that own them.  Reads LDS once per operand
// element and wavefront, against once per output pair on the vector ALUs.
static_assert(kTB == 32 && kBlock == 256, "tile_mma: four wavefronts, each one 16 x 16 block of a 32 x 32 tile");
__device__ __forceinline__ void tile_mma(const Tile &P, const Tile &Q, Tile &Z, double acc[2][2]) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int bi = (w >> 1) * 16, bj = (w & 1) * 16;
    v4d c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < kTB; s4 += 4) {
        const double a = P[bi + (l & 15)][s4 + (l >> 4)];
        const double b = Q[s4 + (l >> 4)][bj + (l & 15)];
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Z[bi + (l >> 4) + 4 * r][bj + (l & 15)] = c[r];
    __syncthreads();
    const int ra = (threadIdx.x / 16) * 2, cb = (threadIdx.x % 16) * 2;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = Z[ra + u][cb + v];
}

// ---- inverse by block Gauss-Jordan sweeps ----
// Sweeping a symmetric matrix on pivot block K (kTB rows) with Q = -(A_KK)^{-1}
// gives A_KK <- Q, A_iK <- -A_iK Q, A_Kj <- -Q A_Kj and A_ij <- A_ij + A_iK Q A_Kj
// for i, j outside K; swept on all of its pivots the matrix becomes -A^{-1}.
// For an SPD matrix each pivot block met is a Schur complement of a leading
// block, SPD as well, so no pivoting is needed, and the matrix stays symmetric:
// only tiles (ti, tj) with ti >= tj are kept (diagonal tiles whole).  A sweep
// reads the matrix from src and writes it to dst in two launches: the pivot
// block column (k_gj_panel: Q and A_iK <- -A_iK Q), then every other tile
// (k_gj_update: A_ij <- A_ij - A_iK' A_Kj with the new A_iK' from the first).
// Tiles of a ragged last block hold the identity on their padded diagonal.

// logical tile (r0 / kTB, c0 / kTB) of the symmetric matrix from stored tile
// (r0, c0) (Tr = false) or, transposed, from stored tile (c0, r0) (Tr = true);
// unconditional loads at clamped indices, zero outside the matrix
template <bool Tr>
__device__ __forceinline__ void tile_load_sym(Tile &T, const double *D, int n, int r0, int c0) {
    const int sr = Tr ? c0 : r0, sc = Tr ? r0 : c0;
#pragma unroll
    for (int e = threadIdx.x; e < kTB * kTB; e += kBlock) {
        const int a = e / kTB, b = e % kTB;
        const double v = D[(size_t)min(sr + a, n - 1) * n + min(sc + b, n - 1)];
        const double w = (sr + a < n && sc + b < n) ? v : 0.0;
        if (Tr) T[b][a] = w;
        else T[a][b] = w;
    }
}

// logical tile (ti, tj) of the symmetric matrix kept as lower tiles
__device__ __forceinline__ void tile_load_lower(Tile &T, const double *D, int n, int ti, int tj) {
    if (ti >= tj) tile_load_sym<false>(T, D, n, ti * kTB, tj * kTB);
    else tile_load_sym<true>(T, D, n, ti * kTB, tj * kTB);
}

__device__ __forceinline__ void tile_from_p(long p, int &ti, int &tj) {
    long i = (long)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > p) --i;
    while ((i + 1) * (i + 2) / 2 <= p) ++i;
    ti = (int)i;
    tj = (int)(p - i * (i + 1) / 2);
}

// Scalar sweeps of a kTB x kTB block held 2 x 2 per thread in q (rows ra, ra+1,
// columns cb, cb+1; exactly symmetric on entry): a_mm <- -1/a_mm,
// a_rm <- a_rm/a_mm, a_rc <- a_rc - a_rm a_mc/a_mm, pivot by pivot, the pivot
// row broadcast through vb in LDS; symmetric products keep the block exactly
// symmetric.  Leaves -block^{-1} in q; a non-positive pivot sets *bad when
// report.  Every thread of the workgroup takes part.
__device__ __forceinline__ void sweep_block(double (&q)[2][2], double (&vb)[2][kTB], int *bad, bool report) {
    const int t = threadIdx.x, ra = (t / 16) * 2, cb = (t % 16) * 2;
    if (ra == 0) {
        vb[0][cb] = q[0][0];
        vb[0][cb + 1] = q[0][1];
    }
    __syncthreads();
    for (int m = 0; m < kTB; ++m) {
        const double *v = vb[m & 1];
        const double piv = v[m];
        if (!(piv > 0.0) && report && t == 0) atomicOr(bad, 1);
        const double rp = 1.0 / piv;
        const double vr[2] = {v[ra], v[ra + 1]}, vc[2] = {v[cb], v[cb + 1]};
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                const int r = ra + u, c = cb + w;
                const double upd = q[u][w] - (vr[u] * vc[w]) * rp;
                q[u][w] = r == m ? (c == m ? -rp : vc[w] * rp) : (c == m ? vr[u] * rp : upd);
            }
        if (m + 1 < kTB && (ra == m + 1 || ra + 1 == m + 1)) {
            const bool lo = ra == m + 1;
            vb[(m + 1) & 1][cb] = lo ? q[0][0] : q[1][0];
            vb[(m + 1) & 1][cb + 1] = lo ? q[0][1] : q[1][1];
        }
        __syncthreads();
    }
}

// Pivot block column of sweep k: Q = -(A_KK)^{-1} from qin (swept by the
// previous update launch) or, for the first pivot block (qin null), swept by
// every workgroup itself while A_iK is loading; then tile row k gets Q and any
// other one -A_iK Q.  One workgroup per tile row.
__global__ __launch_bounds__(kBlock) void k_gj_panel(int n, const double *srcb, double *dstb, int k,
                                                     const double *qin, int *bad) {
    __shared__ Tile X, Qs, Z;
    __shared__ double vb[2][kTB];
    const double *src = bat(srcb, n);
    double *dst = bat(dstb, n);
    const int ti = blockIdx.x;
    const int t = threadIdx.x, ra = (t / 16) * 2, cb = (t % 16) * 2;
    const int K0 = k * kTB;
    double q[2][2];
    if (qin) {
        const double *qz = qin + (size_t)blockIdx.z * kTB * kTB;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) q[u][v] = qz[(ra + u) * kTB + cb + v];
    } else {
        // this thread's 2 x 2 of the pivot block, from its lower half
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int r = ra + u, c = cb + v, i = K0 + max(r, c), j = K0 + min(r, c);
                const double x = src[(size_t)min(i, n - 1) * n + min(j, n - 1)];
                q[u][v] = i < n ? x : (r == c ? 1.0 : 0.0);
            }
    }
    if (ti != k) tile_load_lower(X, src, n, ti, k);
    if (!qin) sweep_block(q, vb, bad, ti == 0);
    double out[2][2];
    if (ti == k) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) out[u][v] = q[u][v];
    } else {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) Qs[ra + u][cb + v] = q[u][v];
        __syncthreads();
        double z[2][2];
        tile_mma(X, Qs, Z, z);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) out[u][v] = -z[u][v];
    }
    // logical tile (ti, k): stored as is below the pivot row, transposed above it
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int i = ti * kTB + ra + u, j = K0 + cb + v;
            if (i < n && j < n) {
                if (ti >= k) dst[(size_t)i * n + j] = out[u][v];
                else dst[(size_t)j * n + i] = out[u][v];
            }
        }
}

// Every tile outside the pivot row and column of sweep k:
// A_ij <- A_ij - A_iK' A_Kj, A_iK' (new, from k_gj_panel) in dst, A_Kj and A_ij
// (old) in src.  Workgroup p serves the p-th lower tile of the matrix with
// tile row and column k taken out, except that workgroup 0 (dispatched first)
// takes the next pivot block, tile (k + 1, k + 1): it also sweeps its new value
// (symmetric from the lower half, identity on a ragged block's padding) into
// qout for the next panel launch.
__global__ __launch_bounds__(kBlock) void k_gj_update(int n, const double *srcb, double *dstb, int k,
                                                      double *qout, int *bad) {
    __shared__ Tile X, Y, Z;
    __shared__ double vb[2][kTB];
    const double *src = bat(srcb, n);
    double *dst = bat(dstb, n);
    const int T0 = (n + kTB - 1) / kTB;
    const long pd = (long)k * (k + 1) / 2 + k;  // tile (k + 1, k + 1) in the reduced numbering
    const bool next = k + 1 < T0;
    long p = blockIdx.x;
    if (next) p = p == 0 ? pd : (p == pd ? 0 : p);
    int ti, tj;
    tile_from_p(p, ti, tj);
    ti += ti >= k;
    tj += tj >= k;
    const int t = threadIdx.x, ra = (t / 16) * 2, cb = (t % 16) * 2;
    tile_load_lower(X, dst, n, ti, k);
    tile_load_lower(Y, src, n, k, tj);
    double a[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int i = ti * kTB + ra + u, j = tj * kTB + cb + v;
            const double x = src[(size_t)min(i, n - 1) * n + min(j, n - 1)];
            a[u][v] = (i < n && j < n) ? x : 0.0;
        }
    __syncthreads();
    double z[2][2];
    tile_mma(X, Y, Z, z);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int i = ti * kTB + ra + u, j = tj * kTB + cb + v;
            a[u][v] -= z[u][v];
            if (i < n && j < n) dst[(size_t)i * n + j] = a[u][v];
        }
    if (!(next && blockIdx.x == 0)) return;  // uniform per workgroup
    __syncthreads();  // every thread is done reading X
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) X[ra + u][cb + v] = a[u][v];
    __syncthreads();
    const int D0 = (k + 1) * kTB;
    double q[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int r = ra + u, c = cb + v;
            q[u][v] = D0 + max(r, c) < n ? X[max(r, c)][min(r, c)] : (r == c ? 1.0 : 0.0);
        }
    sweep_block(q, vb, bad, true);
    double *qz = qout + (size_t)blockIdx.z * kTB * kTB;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) qz[(ra + u) * kTB + cb + v] = q[u][v];
}

// inv = -S for the fully swept S in src (lower tiles): output tile (bx, by) of
// the whole matrix from the lower half, so that inv is exactly symmetric
__global__ __launch_bounds__(kBlock) void k_gj_out(int n, const double *srcb, double *invb) {
    __shared__ Tile T;
    const double *src = bat(srcb, n);
    double *inv = bat(invb, n);
    const int bi = blockIdx.y, bj = blockIdx.x;
    tile_load_lower(T, src, n, bi, bj);
    __syncthreads();
    for (int e = threadIdx.x; e < kTB * kTB; e += kBlock) {
        const int a = e / kTB, b = e % kTB, i = bi * kTB + a, j = bj * kTB + b;
        const double v = (bi == bj && b > a) ? T[b][a] : T[a][b];
        if (i < n && j < n) inv[(size_t)i * n + j] = -v;
    }
}

// sliced-ELL copy of a CSR matrix, one wavefront per slice of 64 rows:
// widths (64 x the longest row of the slice), then the column-major fill
// per slice of 64 rows: 64 x the longest row, the smallest column (rows are
// sorted), a flag when the slice spans 65536 columns or more and one when its
// longest row has more than 8 entries (plain stores of 1: no atomics queue on
// the one address)
__global__ void k_sell_width(int n, int nsl, const int *rp, const int *ci, int *cnt, int *base, int *wide,
                             int *over8) {
    const int lane = threadIdx.x % 64;
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) / 64, nw = gridDim.x * blockDim.x / 64;
    for (int sl = w; sl < nsl; sl += nw) {
        const int r = sl * 64 + lane;
        const int p0 = r < n ? rp[r] : 0, p1 = r < n ? rp[r + 1] : 0;
        int len = p1 - p0;
        int lo = len ? ci[p0] : INT_MAX, hi = len ? ci[p1 - 1] : -1;
        for (int off = 32; off > 0; off >>= 1) {
            len = max(len, __shfl_xor(len, off));
            lo = min(lo, __shfl_xor(lo, off));
            hi = max(hi, __shfl_xor(hi, off));
        }
        if (lane == 0) {
            cnt[sl] = len * 64;
            base[sl] = hi >= lo ? lo : 0;
            if (hi >= lo && hi - lo > 65535) *wide = 1;
            if (len > 8) *over8 = 1;
        }
    }
}

__global__ void k_sell_fill(int n, int nsl, const int *rp, const int *ci, const double *v, const int *soff,
                            const int *base, uint16_t *scd, double *sv) {
    const int lane = threadIdx.x % 64;
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) / 64, nw = gridDim.x * blockDim.x / 64;
    for (int sl = w; sl < nsl; sl += nw) {
        const int r = sl * 64 + lane;
        const int o = soff[sl], wd = (soff[sl + 1] - o) / 64, b = base[sl];
        const int p0 = r < n ? rp[r] : 0, len = r < n ? rp[r + 1] - p0 : 0;
        for (int k = 0; k < wd; ++k) {
            const size_t q = (size_t)o + (size_t)k * 64 + lane;
            scd[q] = (uint16_t)(k < len ? ci[p0 + k] - b : 0);
            sv[q] = k < len ? v[p0 + k] : 0.0;
        }
    }
}

#pragma clang fp contract(off)

// padded FP64 and float32 copies of a dense n x n operator (row stride ld)
__global__ void k_pad_dense(int n, int ld, const double *src, double *d64, float *d32) {
    const long tot = (long)n * ld;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e / ld), k = (int)(e % ld);
        const double v = k < n ? src[(size_t)i * n + k] : 0.0;
        d64[e] = v;
        d32[e] = (float)v;
    }
}

// C = op(A) B, n x n row-major, op(A) = A or A^T; 16x16 LDS tiles
__global__ void k_gemm(int n, const double *A, int transA, const double *B, double *C) {
    __shared__ double ta[16][17], tb[16][17];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
    double acc = 0.0;
    for (int k0 = 0; k0 < n; k0 += 16) {
        const int ka = k0 + tx, kb = k0 + ty;
        double a = 0.0, b = 0.0;
        if (row < n && ka < n) a = transA ? A[(size_t)ka * n + row] : A[(size_t)row * n + ka];
        if (kb < n && col < n) b = B[(size_t)kb * n + col];
        ta[ty][tx] = a;
        tb[ty][tx] = b;
        __syncthreads();
        for (int k = 0; k < 16; ++k) acc += ta[ty][k] * tb[k][tx];
        __syncthreads();
    }
    if (row < n && col < n) C[(size_t)row * n + col] = acc;
}

// H = 1/2 (T + T^T), T = XtY + beta Mu
__global__ void k_hsym(int n, const double *XtY, const double *Mu, double beta, double *H) {
    const long tot = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        const double tij = XtY[(size_t)i * n + j] + beta * Mu[(size_t)i * n + j];
        const double tji = XtY[(size_t)j * n + i] + beta * Mu[(size_t)j * n + i];
        H[e] = 0.5 * (tij + tji);
    }
}

int gsz(long n) {
    long g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

// grid for one wavefront per row
int gwave(long rows) {
    return gsz(rows * 64);
}

// A batch of nb dense inverses of order n (see Setup::plan_dense): the sparse
// inputs (densified into D) or none (D filled by the caller), the work buffers,
// the inverses (back to back) and optionally their padded apply copies.
struct DenseJob {
    int n = 0, nb = 0;
    const DCsr *mats[2] = {nullptr, nullptr};
    double *D = nullptr, *acc = nullptr, *inv = nullptr;
    double *qb = nullptr;  // the next pivot block's -A_KK^{-1}, per matrix
    DenseOp op[2];
    int *bad = nullptr;
};

// The launches of a dense job on stream st: densify, one block Gauss-Jordan
// sweep per pivot block, the inverse out of the swept matrix, apply copies.
// Touches no host state but the job, so it may run on another host thread.
void launch_dense(const DenseJob &j, hipStream_t st) {
    const int n = j.n, nb = j.nb;
    const size_t nn = (size_t)n * n;
    if (j.mats[0]) {
        AMG_HIP(hipMemsetAsync(j.D, 0, sizeof(double) * nb * nn, st));
        for (int b = 0; b < nb; ++b)
            hipLaunchKernelGGL(k_densify, dim3(gwave(n)), dim3(kBlock), 0, st, n, j.mats[b]->rp, j.mats[b]->ci,
                               j.mats[b]->v, (const uint8_t *)nullptr, (const uint8_t *)nullptr, j.D + b * nn);
    }
    // block Gauss-Jordan sweeps, D and acc in turn as source and destination
    const int T0 = ceil_div(n, kTB);
    double *buf[2] = {j.D, j.acc};
    for (int k = 0; k < T0; ++k) {
        hipLaunchKernelGGL(k_gj_panel, dim3(T0, 1, nb), dim3(kBlock), 0, st, n, buf[k & 1], buf[(k + 1) & 1], k,
                           k > 0 ? (const double *)j.qb : nullptr, j.bad);
        if (T0 > 1)
            hipLaunchKernelGGL(k_gj_update, dim3((T0 - 1) * T0 / 2, 1, nb), dim3(kBlock), 0, st, n, buf[k & 1],
                               buf[(k + 1) & 1], k, j.qb, j.bad);
    }
    hipLaunchKernelGGL(k_gj_out, dim3(T0, T0, nb), dim3(kBlock), 0, st, n, buf[T0 & 1], j.inv);
    for (int b = 0; b < nb; ++b)
        if (j.op[b].m64)
            hipLaunchKernelGGL(k_pad_dense, dim3(gsz((long)n * j.op[b].ld)), dim3(kBlock), 0, st, n, j.op[b].ld,
                               j.inv + b * nn, j.op[b].m64, j.op[b].m32);
    AMG_HIP(hipGetLastError());
}

// Host thread that issues the side stream's launches, job after job, so that
// the calling thread keeps feeding the main stream.  A job first makes the
// side stream wait for the event that the calling thread recorded on the
// main stream when it handed the job over.
struct SideWorker {
    std::mutex m;
    std::condition_variable cv;
    std::deque<std::pair<hipEvent_t, DenseJob>> q;
    bool done = false;
    std::thread th;
    hipStream_t st = nullptr;
    int code = 0;
    std::string err;

    void push(hipEvent_t ev, const DenseJob &j) {
        if (!th.joinable()) {
            int dev = 0;
            AMG_HIP(hipGetDevice(&dev));
            th = std::thread([this, dev] { run(dev); });
        }
        {
            std::lock_guard<std::mutex> g(m);
            q.emplace_back(ev, j);
        }
        cv.notify_one();
    }
    void run(int dev) {
        (void)hipSetDevice(dev);
        for (;;) {
            std::pair<hipEvent_t, DenseJob> job;
            {
                std::unique_lock<std::mutex> lk(m);
                cv.wait(lk, [&] { return done || !q.empty(); });
                if (q.empty()) return;
                job = q.front();
                q.pop_front();
            }
            if (code) continue;  // after a failure the rest is skipped
            try {
                AMG_HIP(hipStreamWaitEvent(st, job.first, 0));
                launch_dense(job.second, st);
            } catch (const Error &e) {
                code = e.code;
                err = e.msg;
            }
        }
    }
    // every job issued (the thread ends); reports the first failure
    void finish() {
        stop();
        if (code) fail(code, err);
    }
    void stop() {
        {
            std::lock_guard<std::mutex> g(m);
            done = true;
        }
        cv.notify_one();
        if (th.joinable()) th.join();
    }
    ~SideWorker() { stop(); }
};

struct Setup {
    Ctx &c;
    hipStream_t s;
    // scratch words of this stream's sparse products and scans (device, pinned host)
    int *isc;
    int *hisc;
    // when set, released blocks wait here until the caller has joined the streams
    std::vector<void *> *defer = nullptr;
    explicit Setup(Ctx &cc) : c(cc), s(cc.stream), isc(cc.iscratch), hisc(cc.hiscr) {}
    Setup(Ctx &cc, hipStream_t st) : c(cc), s(st), isc(cc.iscratch), hisc(cc.hiscr) {}
    Setup(Ctx &cc, hipStream_t st, int *is, int *his, std::vector<void *> *df)
        : c(cc), s(st), isc(is), hisc(his), defer(df) {}

    void rel(void *p) {
        if (defer) defer->push_back(p);
        else c.arena.release(p);
    }

    int read_int(const int *d) {
        AMG_HIP(hipMemcpyAsync(hisc, d, sizeof(int), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        return hisc[0];
    }

    void zero(void *p, size_t bytes) { AMG_HIP(hipMemsetAsync(p, 0, bytes, s)); }

    // Sticky failure flags of checks that need no immediate answer (nothing
    // downstream indexes memory by the flagged values): set by kernels,
    // cleared once per phase and read at its end in one transfer.
    static constexpr int kFlag0 = 16, kFlagN = 32;
    static constexpr int kFlagFill = 16, kFlagMirror = 17, kFlagPivot = 18, kFlagMassDiag = 19, kFlagDiag = 20;
    static constexpr int kFlagAlign = kFlag0 + kFlagN - 1;  // the level flags end before it
    static constexpr int kFlagDiagN = kFlagAlign - kFlagDiag;
    void clear_flags() { zero(c.iscratch + kFlag0, kFlagN * sizeof(int)); }
    void check_flags() {
        AMG_HIP(hipMemcpyAsync(c.hiscr, c.iscratch + kFlag0, kFlagN * sizeof(int), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        const int *f = c.hiscr - kFlag0;
        for (int j = 0; j < kFlagDiagN; ++j)
            if (f[kFlagDiag + j]) fail(AMG_ERR_NOT_SPD, "non-positive diagonal at level " + std::to_string(j));
        if (f[kFlagAlign]) fail(AMG_ERR_ARG, "prolongator entry missing from A S");
        if (f[kFlagMassDiag]) fail(AMG_ERR_NOT_SPD, "mass matrix has a non-positive diagonal");
        if (f[kFlagPivot]) fail(AMG_ERR_NOT_SPD, "dense inverse met a non-positive pivot");
        if (f[kFlagMirror]) fail(AMG_ERR_ARG, "coarse matrix pattern is not symmetric");
        if (f[kFlagFill]) fail(AMG_ERR_CAPACITY, "sparse product: output column lost in the fill");
    }

    // out[0..n] exclusive scan of cnt[0..n-1]; the total is left in isc[8]
    // and returned when read (else -1: no wait for the device)
    int scan(const int *cnt, int *out, int n, bool read = true) {
        const int nb = std::max(1, ceil_div(n, kScanPer));
        int *bsum = c.arena.alloc<int>(nb);
        if (n > 0) hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kBlock), 0, s, n, cnt, bsum);
        hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kBlock), 0, s, n, nb, cnt, bsum, out, isc + 8);
        const int total = read ? read_int(isc + 8) : -1;
        rel(bsum);
        return total;
    }

    void check_kernels() { AMG_HIP(hipGetLastError()); }

    DCsr copy_in(const amg_csr &m) {
        DCsr d;
        d.n = m.nrows;
        d.m = m.ncols;
        d.nnz = m.nnz;
        d.rp = c.arena.alloc<int>(d.n + 1);
        d.ci = c.arena.alloc<int>(d.nnz);
        d.v = c.arena.alloc<double>(d.nnz);
        AMG_HIP(hipMemcpyAsync(d.rp, m.rowptr, sizeof(int) * (d.n + 1), hipMemcpyDefault, s));
        AMG_HIP(hipMemcpyAsync(d.ci, m.col, sizeof(int) * d.nnz, hipMemcpyDefault, s));
        AMG_HIP(hipMemcpyAsync(d.v, m.val, sizeof(double) * d.nnz, hipMemcpyDefault, s));
        return d;
    }

    void check_matrix(const DCsr &d, const char *name) {
        zero(c.iscratch, 2 * sizeof(int));
        hipLaunchKernelGGL(k_check_sym, dim3(gsz((long)(d.n) * kRowLanes)), dim3(kBlock), 0, s, d.n, d.rp, d.ci, d.v, c.iscratch);
        check_kernels();
        AMG_HIP(hipMemcpyAsync(c.hiscr, c.iscratch, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        if (c.hiscr[1]) fail(AMG_ERR_ARG, std::string(name) + ": columns not sorted/unique within a row");
        if (c.hiscr[0]) fail(AMG_ERR_NOT_SYMMETRIC, std::string(name) + " is not exactly symmetric");
    }

    // A sparse product in three phases so that two can run on two streams with
    // one wait between them: prod_count issues the symbolic pass, the scan and
    // the read of its results without waiting; prod_wait waits (and counts
    // again the rows that overflowed the first tier); prod_fill allocates the
    // output and issues the numeric pass.
    struct Prod {
        const DCsr *A = nullptr, *B = nullptr;
        DCsr C;
        int *cnt = nullptr;
        bool wide = false;
        int dc = 0;  // > 0: B has at most dc columns, dense-accumulator passes
        int gr = 0, umax = 0, bmax = 0;
    };

    Prod prod_count(const DCsr &A, const DCsr &B) {
        Prod pr;
        pr.A = &A;
        pr.B = &B;
        DCsr &C = pr.C;
        C.n = A.n;
        C.m = B.m;
        pr.cnt = c.arena.alloc<int>(A.n + 1);
        C.rp = c.arena.alloc<int>(A.n + 1);
        int *cnt = pr.cnt;
        zero(isc + 4, sizeof(int));
        zero(isc + 10, 3 * sizeof(int));
        // rows too few to fill the chip: four wavefronts per row; otherwise
        // groups of 16, 32 or 64 lanes per row, from the mean row length of A
        const bool wide = pr.wide = A.n < 8192;
        const int gr = pr.gr = std::max(1, std::min(A.n, 32768));
        const long mean = ceil_div(A.nnz, std::max(1, A.n));
        const int lpr = mean <= 16 ? 16 : mean <= 32 ? 32 : 64;
        const int grs = std::max(1, std::min(ceil_div(A.n, kBlock / lpr), 4096));
        auto count = [&](auto kern, int recount) {
            hipLaunchKernelGGL(kern, dim3(gr), dim3(wide ? 256 : 64), 0, s, A.n, A.rp, A.ci, B.rp, B.ci, cnt,
                               isc + 4, isc + 10, recount);
        };
        auto count_sub = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(grs), dim3(kBlock), 0, s, A.n, A.rp, A.ci, B.rp, B.ci, cnt, isc + 10);
        };
        // dense accumulators for the products of few rows whose B has at most
        // 2048 columns (for many rows the hash passes are faster)
        pr.dc = !wide ? 0 : B.m <= 256 ? 256 : B.m <= 512 ? 512 : B.m <= 1024 ? 1024 : B.m <= 2048 ? 2048 : 0;
        auto count_dense = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(std::max(1, std::min(A.n, 65535))), dim3(64), 0, s, A.n, A.rp, A.ci, B.rp,
                               B.ci, cnt, isc + 10);
        };
        // first tier: small tables; rows that overflow half of one are counted
        // again with kHS slots
        if (pr.dc == 256) count_dense(k_spgemm_count_dense<256>);
        else if (pr.dc == 512) count_dense(k_spgemm_count_dense<512>);
        else if (pr.dc == 1024) count_dense(k_spgemm_count_dense<1024>);
        else if (pr.dc == 2048) count_dense(k_spgemm_count_dense<2048>);
        else if (wide) count(k_spgemm_count<4, 512>, 0);
        else if (lpr == 16) count_sub(k_spgemm_count_sub<16, 128>);
        else if (lpr == 32) count_sub(k_spgemm_count_sub<32, 256>);
        else count_sub(k_spgemm_count_sub<64, 512>);
        check_kernels();
        // the row offsets before the one read of the pass's results: the
        // total (isc[8]) arrives with the maxima (a row counted again makes
        // the first scan moot and it is redone)
        scan(cnt, C.rp, A.n, false);
        AMG_HIP(hipMemcpyAsync(hisc, isc + 4, 9 * sizeof(int), hipMemcpyDeviceToHost, s));
        return pr;
    }

    void prod_wait(Prod &pr) {
        const DCsr &A = *pr.A, &B = *pr.B;
        AMG_HIP(hipStreamSynchronize(s));
        if (hisc[8]) {
            if (pr.wide)
                hipLaunchKernelGGL((k_spgemm_count<4, kHS>), dim3(pr.gr), dim3(256), 0, s, A.n, A.rp, A.ci, B.rp,
                                   B.ci, pr.cnt, isc + 4, isc + 10, 1);
            else
                hipLaunchKernelGGL((k_spgemm_count<1, kHS>), dim3(pr.gr), dim3(64), 0, s, A.n, A.rp, A.ci, B.rp,
                                   B.ci, pr.cnt, isc + 4, isc + 10, 1);
            check_kernels();
            scan(pr.cnt, pr.C.rp, A.n, false);
            AMG_HIP(hipMemcpyAsync(hisc, isc + 4, 9 * sizeof(int), hipMemcpyDeviceToHost, s));
            AMG_HIP(hipStreamSynchronize(s));
        }
        if (hisc[0])
            fail(AMG_ERR_CAPACITY, "sparse product row exceeds " + std::to_string(kMaxRowOut) + " columns");
        pr.umax = hisc[6];
        pr.bmax = hisc[7];
        pr.C.nnz = hisc[4];
    }

    DCsr prod_fill(Prod &pr) {
        const DCsr &A = *pr.A, &B = *pr.B;
        DCsr &C = pr.C;
        const bool wide = pr.wide;
        const int gr = pr.gr, umax = pr.umax, bmax = pr.bmax;
        C.ci = c.arena.alloc<int>(C.nnz);
        C.v = c.arena.alloc<double>(C.nnz);
        if (C.nnz == 0) {  // no products: the numeric kernels assume B has entries
            rel(pr.cnt);
            return C;
        }
        if (pr.dc > 0) {
            // four wavefronts per row when rows of B are longer than one wavefront
            const int nw = bmax > 64 ? 4 : 1;
            auto fill = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(std::max(1, std::min(A.n, 65535))), dim3(64 * nw), 0, s, A.n, B.m,
                                   A.rp, A.ci, A.v, B.rp, B.ci, B.v, C.rp, C.ci, C.v);
            };
            if (nw == 1) {
                if (pr.dc == 256) fill(k_spgemm_fill_dense<256, 1>);
                else if (pr.dc == 512) fill(k_spgemm_fill_dense<512, 1>);
                else if (pr.dc == 1024) fill(k_spgemm_fill_dense<1024, 1>);
                else fill(k_spgemm_fill_dense<2048, 1>);
            } else {
                if (pr.dc == 256) fill(k_spgemm_fill_dense<256, 4>);
                else if (pr.dc == 512) fill(k_spgemm_fill_dense<512, 4>);
                else if (pr.dc == 1024) fill(k_spgemm_fill_dense<1024, 4>);
                else fill(k_spgemm_fill_dense<2048, 4>);
            }
        } else if (wide) {
            // G rows of B per step when every row of B fits 256 / G threads (groups of 8 at least)
            int G = 1;
            while (2 * G <= 256 / 8 && 256 / (2 * G) >= bmax) G *= 2;
            auto fill = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(gr), dim3(256), 0, s, A.n, G, A.rp, A.ci, A.v, B.rp, B.ci, B.v, C.rp,
                                   C.ci, C.v, c.iscratch + kFlagFill);
            };
            if (umax <= 128) fill(k_spgemm_fill<256, 4>);
            else if (umax <= 256) fill(k_spgemm_fill<512, 4>);
            else if (umax <= 512) fill(k_spgemm_fill<1024, 4>);
            else fill(k_spgemm_fill<2048, 4>);
        } else if (umax <= 256) {
            // BL lanes per row of B (a power of two from 8 to 64); at least 16
            // lanes per row of A, 32 with the largest tables (LDS per workgroup
            // 14 HS kBlock / LPR bytes, at most 56 KiB)
            const int bl = bmax <= 8 ? 8 : bmax <= 16 ? 16 : bmax <= 32 ? 32 : 64;
            const int hs = umax <= 32 ? 64 : umax <= 64 ? 128 : umax <= 128 ? 256 : 512;
            const int fl = std::max(hs == 512 ? 32 : 16, bl);
            const int grf = std::max(1, std::min(ceil_div(A.n, kBlock / fl), 16384));
            auto fill = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(grf), dim3(kBlock), 0, s, A.n, A.rp, A.ci, A.v, B.rp, B.ci, B.v, C.rp,
                                   C.ci, C.v, c.iscratch + kFlagFill);
            };
            const int key = fl * 10000 + hs * 10 + bl / 8;
            switch (key) {
            case 160641: fill(k_spgemm_fill_sub<16, 64, 8>); break;
            case 161281: fill(k_spgemm_fill_sub<16, 128, 8>); break;
            case 162561: fill(k_spgemm_fill_sub<16, 256, 8>); break;
            case 325121: fill(k_spgemm_fill_sub<32, 512, 8>); break;
            case 160642: fill(k_spgemm_fill_sub<16, 64, 16>); break;
            case 161282: fill(k_spgemm_fill_sub<16, 128, 16>); break;
            case 162562: fill(k_spgemm_fill_sub<16, 256, 16>); break;
            case 325122: fill(k_spgemm_fill_sub<32, 512, 16>); break;
            case 320644: fill(k_spgemm_fill_sub<32, 64, 32>); break;
            case 321284: fill(k_spgemm_fill_sub<32, 128, 32>); break;
            case 322564: fill(k_spgemm_fill_sub<32, 256, 32>); break;
            case 325124: fill(k_spgemm_fill_sub<32, 512, 32>); break;
            case 640648: fill(k_spgemm_fill_sub<64, 64, 64>); break;
            case 641288: fill(k_spgemm_fill_sub<64, 128, 64>); break;
            case 642568: fill(k_spgemm_fill_sub<64, 256, 64>); break;
            case 645128: fill(k_spgemm_fill_sub<64, 512, 64>); break;
            default: fail(AMG_ERR_HIP, "sparse product: no fill kernel for this shape");
            }
        } else {
            int G = 1;
            while (2 * G <= 64 / 8 && 64 / (2 * G) >= bmax) G *= 2;
            auto fill = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(gr), dim3(64), 0, s, A.n, G, A.rp, A.ci, A.v, B.rp, B.ci, B.v, C.rp,
                                   C.ci, C.v, c.iscratch + kFlagFill);
            };
            if (umax <= 512) fill(k_spgemm_fill<1024, 1>);
            else fill(k_spgemm_fill<2048, 1>);
        }
        check_kernels();
        rel(pr.cnt);
        return C;
    }

    DCsr spgemm(const DCsr &A, const DCsr &B) {
        Prod pr = prod_count(A, B);
        prod_wait(pr);
        return prod_fill(pr);
    }

    DCsr transpose(const DCsr &A) {
        DCsr T;
        T.n = A.m;
        T.m = A.n;
        T.nnz = A.nnz;
        T.rp = c.arena.alloc<int>(T.n + 1);
        T.ci = c.arena.alloc<int>(T.nnz);
        T.v = c.arena.alloc<double>(T.nnz);
        if (T.n <= kTbCols && A.n > 0) {
            const int nb = ceil_div(A.n, kTbRows);
            const long len = (long)T.n * nb;
            if (len < (long)INT_MAX) {
                int *hist = c.arena.alloc<int>(len);
                int *pos = c.arena.alloc<int>(len + 1);
                hipLaunchKernelGGL(k_tb_hist, dim3(nb), dim3(kBlock), 0, s, A.n, T.n, nb, A.rp, A.ci, hist);
                scan(hist, pos, (int)len, false);  // the total is A.nnz
                hipLaunchKernelGGL(k_tb_place, dim3(nb), dim3(kBlock), 0, s, A.n, T.n, nb, A.rp, A.ci, A.v, pos,
                                   T.rp, T.ci, T.v);
                check_kernels();
                c.arena.release(hist);
                c.arena.release(pos);
                return T;
            }
        }
        int *cnt = c.arena.alloc<int>(T.n + 1);
        int *fill = c.arena.alloc<int>(T.n + 1);
        zero(cnt, sizeof(int) * (T.n + 1));
        zero(fill, sizeof(int) * (T.n + 1));
        int *tci = c.arena.alloc<int>(T.nnz);
        double *tv = c.arena.alloc<double>(T.nnz);
        hipLaunchKernelGGL(k_t_count, dim3(gsz(A.n)), dim3(kBlock), 0, s, A.n, A.rp, A.ci, cnt);
        scan(cnt, T.rp, T.n, false);  // the total is A.nnz
        hipLaunchKernelGGL(k_t_place, dim3(gsz(A.n)), dim3(kBlock), 0, s, A.n, A.rp, A.ci, A.v, T.rp, fill, tci,
                           tv);
        const int waves_g = std::min(4096, std::max(1, ceil_div(T.n, 4)));
        hipLaunchKernelGGL(k_row_sort, dim3(waves_g), dim3(kBlock), 0, s, T.n, T.rp, tci, tv, T.ci, T.v);
        check_kernels();
        c.arena.release(cnt);
        c.arena.release(fill);
        c.arena.release(tci);
        c.arena.release(tv);
        return T;
    }

    // The Galerkin products of A (this stream) and M (the context's second
    // setup stream, with its own scratch words) side by side: the products run
    // in pairs whose count read-backs share one wait, the M side starts behind
    // everything issued here so far, and every block released meanwhile (by
    // either side) returns to the arena only after this stream has joined the
    // other.  With keep, A S is handed back.
    void galerkin_pair(const DCsr &S, const DCsr &St, const DCsr &A, const DCsr &M, DCsr &CA, DCsr &CM,
                       DCsr *keep) {
        std::vector<void *> deferred;
        Setup g(c, c.gal, c.iscratch2, c.hiscr2, &deferred);
        std::vector<void *> *saved = defer;
        defer = &deferred;
        AMG_HIP(hipEventRecord(c.gal_ev[0], s));
        AMG_HIP(hipStreamWaitEvent(c.gal, c.gal_ev[0], 0));
        Prod pa = prod_count(A, S), pm = g.prod_count(M, S);
        prod_wait(pa);
        g.prod_wait(pm);
        DCsr TA = prod_fill(pa), TM = g.prod_fill(pm);
        Prod qa = prod_count(St, TA), qm = g.prod_count(St, TM);
        prod_wait(qa);
        g.prod_wait(qm);
        CA = prod_fill(qa);
        CM = g.prod_fill(qm);
        hipLaunchKernelGGL(k_mirror, dim3(gwave(CA.n)), dim3(kBlock), 0, s, CA.n, CA.rp, CA.ci, CA.v,
                           c.iscratch + kFlagMirror);
        hipLaunchKernelGGL(k_mirror, dim3(gwave(CM.n)), dim3(kBlock), 0, c.gal, CM.n, CM.rp, CM.ci, CM.v,
                           c.iscratch + kFlagMirror);
        check_kernels();
        for (void *p : {(void *)TM.rp, (void *)TM.ci, (void *)TM.v}) deferred.push_back(p);
        if (keep) *keep = TA;
        else
            for (void *p : {(void *)TA.rp, (void *)TA.ci, (void *)TA.v}) deferred.push_back(p);
        AMG_HIP(hipEventRecord(c.gal_ev[1], c.gal));
        AMG_HIP(hipStreamWaitEvent(s, c.gal_ev[1], 0));
        defer = saved;
        for (void *p : deferred) rel(p);
    }

    // returns false when coarsening stops at level j
    bool coarsen(int j) {
        Level &L0 = c.lev[j];
        const DCsr &A = L0.A;
        const int n = A.n;
        const uint8_t *mask = L0.mask;
        double *d = c.arena.alloc<double>(n);
        hipLaunchKernelGGL(k_diag, dim3(gsz((long)(n) * kRowLanes)), dim3(kBlock), 0, s, n, A.rp, A.ci, A.v, mask, d,
                           c.iscratch + kFlagDiag + std::min(j, kFlagDiagN - 1));
        // the input matrix is checked before anything is built on it
        if (j == 0 && read_int(c.iscratch + kFlagDiag))
            fail(AMG_ERR_NOT_SPD, "non-positive diagonal at level 0");
        // strength graph
        const double theta = c.o.theta0 * std::ldexp(1.0, -j);
        const double t = theta * theta;
        uint8_t *flag = c.arena.alloc<uint8_t>(A.nnz);
        int *cnt = c.arena.alloc<int>(n + 1);
        int *srp = c.arena.alloc<int>(n + 1);
        hipLaunchKernelGGL(k_strength, dim3(gsz((long)(n) * kRowLanes)), dim3(kBlock), 0, s, n, A.rp, A.ci, A.v, d, mask, t, flag,
                           cnt);
        // the strong entries are a subset of A's: A.nnz bounds them with no
        // wait for the count
        scan(cnt, srp, n, false);
        int *sci = c.arena.alloc<int>(A.nnz);
        double *sabs = c.arena.alloc<double>(A.nnz);
        hipLaunchKernelGGL(k_strong_fill, dim3(gsz((long)(n) * kRowLanes)), dim3(kBlock), 0, s, n, A.rp, A.ci, A.v, flag, srp, sci,
                           sabs);
        c.arena.release(flag);
        // distance-2 independent set by fixed-priority rounds
        uint64_t *h = c.arena.alloc<uint64_t>(n);
        const uint64_t base = c.o.agg_seed ^ ((uint64_t)j << 40);
        hipLaunchKernelGGL(k_hash, dim3(gsz(n)), dim3(kBlock), 0, s, n, base, h);
        int8_t *st = c.arena.alloc<int8_t>(n);
        int *m1 = c.arena.alloc<int>(n);
        uint8_t *r1 = c.arena.alloc<uint8_t>(n);
        hipLaunchKernelGGL(k_mis_init, dim3(gsz(n)), dim3(kBlock), 0, s, n, mask, st);
        // rounds in batches with one read of the undecided flag per batch;
        // round r leaves a nonzero und[r % kMisRing] while nodes are undecided
        // (the ring holds whole batches)
        constexpr int kMisRing = 64, kMisBatch = 4;
        static_assert(kMisRing % kMisBatch == 0, "a batch must not wrap the ring");
        int *und = c.arena.alloc<int>(kMisRing);
        for (int round = 0;;) {
            if (round > n + 1) fail(AMG_ERR_ARG, "independent-set rounds did not terminate");
            zero(und + round % kMisRing, kMisBatch * sizeof(int));
            for (int b = 0; b < kMisBatch; ++b, ++round) {
                const int *prev = round ? und + (round - 1) % kMisRing : nullptr;
                hipLaunchKernelGGL(k_mis_m1, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, h, st, m1, prev);
                hipLaunchKernelGGL(k_mis_m2, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, h, m1, st, prev);
                hipLaunchKernelGGL(k_mis_r1, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, st, r1, prev);
                hipLaunchKernelGGL(k_mis_r2, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, r1, st,
                                   und + round % kMisRing, prev);
            }
            check_kernels();
            if (read_int(und + (round - 1) % kMisRing) == 0) break;
        }
        c.arena.release(und);
        L0.root = c.arena.alloc<uint8_t>(n);
        int *cid = c.arena.alloc<int>(n + 1);
        hipLaunchKernelGGL(k_root_flags, dim3(gsz(n)), dim3(kBlock), 0, s, n, st, L0.root, cnt);
        scan(cnt, cid, n, false);  // the aggregate count stays in isc[8], read with the check below
        L0.agg = c.arena.alloc<int>(n);
        uint8_t *p2 = c.arena.alloc<uint8_t>(n);
        hipLaunchKernelGGL(k_phase2, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, sabs, L0.root, cid, mask,
                           L0.agg, p2);
        zero(isc + 7, sizeof(int));
        hipLaunchKernelGGL(k_phase3, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, sabs, p2, L0.agg, isc + 7);
        check_kernels();
        AMG_HIP(hipMemcpyAsync(hisc + 7, isc + 7, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        if (hisc[7]) fail(AMG_ERR_ARG, "aggregation left a node unassigned");
        const int nc = hisc[8];
        for (void *p : {(void *)h, (void *)st, (void *)m1, (void *)r1, (void *)p2, (void *)sci, (void *)sabs,
                        (void *)srp, (void *)cid})
            c.arena.release(p);
        if (nc == 0 || (double)nc > 0.9 * (double)n) {
            c.arena.release(cnt);
            c.arena.release(d);
            return false;
        }
        // omega = (4/3) / max_i (sum_k |a_ik|) / a_ii
        double *dl1 = c.arena.alloc<double>(n);
        hipLaunchKernelGGL(k_l1, dim3(gsz((long)(n) * kRowLanes)), dim3(kBlock), 0, s, n, A.rp, A.v, L0.dl1inv, dl1);
        unsigned long long *mb = reinterpret_cast<unsigned long long *>(c.dscratch);
        zero(mb, sizeof(unsigned long long));
        hipLaunchKernelGGL(k_rho, dim3(gsz(n)), dim3(kBlock), 0, s, n, dl1, d, mask, mb);
        check_kernels();
        c.arena.release(dl1);
        // tentative prolongator, then S = (I - omega D^{-1} A) P_tent
        DCsr P;
        P.n = n;
        P.m = nc;
        P.rp = c.arena.alloc<int>(n + 1);
        hipLaunchKernelGGL(k_ptent_count, dim3(gsz(n)), dim3(kBlock), 0, s, n, L0.agg, cnt);
        scan(cnt, P.rp, n, false);
        P.nnz = n;  // at most one entry per row: an upper bound is enough here
        P.ci = c.arena.alloc<int>(P.nnz);
        P.v = c.arena.alloc<double>(P.nnz);
        hipLaunchKernelGGL(k_ptent_fill, dim3(gsz(n)), dim3(kBlock), 0, s, n, L0.agg, P.rp, P.ci, P.v);
        DCsr S = spgemm(A, P);
        hipLaunchKernelGGL(k_smooth, dim3(gsz(n)), dim3(kBlock), 0, s, n, S.rp, S.ci, S.v, L0.agg, d,
                           (const unsigned long long *)mb);
        check_kernels();
        for (void *p : {(void *)P.rp, (void *)P.ci, (void *)P.v, (void *)cnt, (void *)d}) c.arena.release(p);
        L0.S = S;
        L0.St = transpose(S);
        Level nx;
        nx.n = nc;
        galerkin_pair(L0.S, L0.St, A, L0.M, nx.A, nx.M, &L0.T);
        c.lev.push_back(nx);
        return true;
    }

    void level_diag(Level &L) {
        const int n = L.A.n;
        L.n = n;
        if (!L.dl1inv) L.dl1inv = c.arena.alloc<double>(n);
        double *dl1 = c.arena.alloc<double>(n);
        hipLaunchKernelGGL(k_l1, dim3(gsz((long)(n) * kRowLanes)), dim3(kBlock), 0, s, n, L.A.rp, L.A.v, L.dl1inv, dl1);
        double *md = c.arena.alloc<double>(n);
        L.mdinv = c.arena.alloc<double>(n);
        hipLaunchKernelGGL(k_diag, dim3(gsz((long)(n) * kRowLanes)), dim3(kBlock), 0, s, n, L.M.rp, L.M.ci, L.M.v,
                           (const uint8_t *)nullptr, md, c.iscratch + kFlagMassDiag);
        hipLaunchKernelGGL(k_inv, dim3(gsz(n)), dim3(kBlock), 0, s, n, md, L.mdinv);
        check_kernels();
        c.arena.release(dl1);
        c.arena.release(md);
    }

    void make_sell(DCsr &A) {
        const int nsl = ceil_div(A.n, 64);
        int *cnt = c.arena.alloc<int>(nsl + 1);
        int *off = c.arena.alloc<int>(nsl + 1);
        int *base = c.arena.alloc<int>(nsl);
        zero(isc + 13, 2 * sizeof(int));
        hipLaunchKernelGGL(k_sell_width, dim3(gwave(nsl)), dim3(kBlock), 0, s, A.n, nsl, A.rp, A.ci, cnt, base,
                           isc + 13, isc + 14);
        scan(cnt, off, nsl, false);
        // the total (isc[8]) and the flags of a wide slice (isc[13]) and of a
        // slice wider than 8 entries (isc[14]) in one read
        AMG_HIP(hipMemcpyAsync(hisc + 8, isc + 8, 7 * sizeof(int), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        const int tot = hisc[8];
        c.arena.release(cnt);
        if (hisc[13]) {  // 16-bit column offsets do not reach: the CSR kernels serve this matrix
            c.arena.release(off);
            c.arena.release(base);
            return;
        }
        A.sl_off = off;
        A.sl_base = base;
        A.sl_over8 = hisc[14] != 0;
        A.sl_cd = c.arena.alloc<uint16_t>(tot);
        A.sl_v = c.arena.alloc<double>(tot);
        hipLaunchKernelGGL(k_sell_fill, dim3(gwave(nsl)), dim3(kBlock), 0, s, A.n, nsl, A.rp, A.ci, A.v, A.sl_off,
                           A.sl_base, A.sl_cd, A.sl_v);
        if (A.v32) {
            A.sl_v32 = c.arena.alloc<float>(tot);
            hipLaunchKernelGGL(k_to_f32, dim3(gsz(tot)), dim3(kBlock), 0, s, (long)tot, A.sl_v, A.sl_v32);
        }
        A.nsl = nsl;
        check_kernels();
    }

    DenseOp dense_op(const double *inv, int n) {
        DenseOp d;
        d.n = n;
        d.ld = ceil_div(n, 64) * 64;
        d.m64 = c.arena.alloc<double>((size_t)n * d.ld);
        d.m32 = c.arena.alloc<float>((size_t)n * d.ld);
        hipLaunchKernelGGL(k_pad_dense, dim3(gsz((long)n * d.ld)), dim3(kBlock), 0, s, n, d.ld, inv, d.m64, d.m32);
        return d;
    }

    // A batch of dense inverses: its buffers come from the arena here, on the
    // calling thread; launch_dense issues its work on any stream, from any
    // host thread.
    DenseJob plan_dense(std::initializer_list<const DCsr *> mats, bool ops) {
        DenseJob j;
        j.nb = (int)mats.size();
        j.n = (*mats.begin())->n;
        int b = 0;
        for (const DCsr *A : mats) j.mats[b++] = A;
        j.D = c.arena.alloc<double>((size_t)j.nb * j.n * j.n);
        plan_rest(j, ops);
        return j;
    }
    DenseJob plan_factor(double *D, int n) {  // D holds the matrix already
        DenseJob j;
        j.nb = 1;
        j.n = n;
        j.D = D;
        plan_rest(j, false);
        return j;
    }
    void plan_rest(DenseJob &j, bool ops) {
        const size_t nn = (size_t)j.n * j.n;
        j.acc = c.arena.alloc<double>(j.nb * nn);
        j.qb = c.arena.alloc<double>((size_t)j.nb * kTB * kTB);
        j.inv = c.arena.alloc<double>(j.nb * nn);
        j.bad = c.iscratch + kFlagPivot;
        if (ops)
            for (int b = 0; b < j.nb; ++b) {
                DenseOp &d = j.op[b];
                d.n = j.n;
                d.ld = ceil_div(j.n, 64) * 64;
                d.m64 = c.arena.alloc<double>((size_t)j.n * d.ld);
                d.m32 = c.arena.alloc<float>((size_t)j.n * d.ld);
            }
    }
    // the temporaries (D included) back to the arena, or to *defer when the
    // work runs on a stream that the arena's reuse does not follow
    void release_job(DenseJob &j, std::vector<void *> *defer) {
        for (void *p : {(void *)j.D, (void *)j.acc, (void *)j.qb}) {
            if (defer) defer->push_back(p);
            else c.arena.release(p);
        }
    }

    // dense inverses of nb sparse SPD matrices of one order, returned back to
    // back (inverse b at the result + b * n * n), on this stream
    double *dense_inverse(std::initializer_list<const DCsr *> mats) {
        DenseJob j = plan_dense(mats, false);
        launch_dense(j, s);
        release_job(j, nullptr);
        return j.inv;
    }

    // inverse of the SPD matrix in D (overwritten by its factor)
    double *factor_invert(double *D, int n) {
        DenseJob j = plan_factor(D, n);
        launch_dense(j, s);
        release_job(j, nullptr);
        return j.inv;
    }
};

}  // namespace

void build_hierarchy(Ctx &c, const amg_csr &Ain, const amg_csr &Min, const uint8_t *dirichlet) {
    Setup su(c);
    hipStream_t s = c.stream;
    su.clear_flags();
    const int N = Ain.nrows;
    c.N = N;
    DCsr A = su.copy_in(Ain);
    su.check_matrix(A, "A");
    DCsr M = su.copy_in(Min);
    su.check_matrix(M, "M");
    // Dirichlet reduction of the stiffness matrix
    Level l0;
    l0.n = N;
    l0.M = M;
    if (dirichlet) {
        c.mask0 = c.arena.alloc<uint8_t>(N);
        AMG_HIP(hipMemcpyAsync(c.mask0, dirichlet, N, hipMemcpyDefault, s));
        c.has_mask = true;
        l0.mask = c.mask0;
    }
    {
        // the Dirichlet reduction, which also drops A's stored zeros (on the
        // uniform meshes every diagonal edge of a cube's tetrahedra carries
        // exactly zero stiffness: half of the stored entries)
        DCsr A0;
        A0.n = A0.m = N;
        int *cnt = c.arena.alloc<int>(N + 1);
        A0.rp = c.arena.alloc<int>(N + 1);
        hipLaunchKernelGGL(k_a0_count, dim3(gsz((long)(N) * kRowLanes)), dim3(kBlock), 0, s, N, A.rp, A.ci, A.v,
                           c.mask0, cnt);
        A0.nnz = su.scan(cnt, A0.rp, N);
        A0.ci = c.arena.alloc<int>(A0.nnz);
        A0.v = c.arena.alloc<double>(A0.nnz);
        hipLaunchKernelGGL(k_a0_fill, dim3(gsz((long)(N) * kRowLanes)), dim3(kBlock), 0, s, N, A.rp, A.ci, A.v, c.mask0, A0.rp,
                           A0.ci, A0.v);
        su.check_kernels();
        c.arena.release(cnt);
        c.arena.release(A.rp);
        c.arena.release(A.ci);
        c.arena.release(A.v);
        l0.A = A0;
    }
    c.lev.clear();
    c.lev.push_back(l0);
    // The dense inverses of small levels (j >= 1, at most dense_solve_max rows)
    // are built on a side stream as soon as the level exists, while the main
    // stream builds the levels below it.  The side stream starts behind
    // everything queued on the main stream so far (the arena may hand it
    // blocks released there), allocates only when it is started, and its
    // temporaries return to the arena only after the main stream has joined it.
    struct Early {
        double *inv = nullptr;
        DenseOp dA, dM;
    };
    std::vector<Early> early(c.lev.capacity());
    std::vector<void *> deferred;
    struct EvList {  // destroyed after the worker below has ended
        std::vector<hipEvent_t> v;
        ~EvList() {
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
        }
    } fork_ev;
    SideWorker side;
    side.st = c.side;
    auto fork_dense = [&](int jl) {  // A_j^{-1} and M_j^{-1}
        Level &Lv = c.lev[jl];
        DenseJob job = su.plan_dense({&Lv.A, &Lv.M}, true);
        hipEvent_t ev = nullptr;
        AMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        fork_ev.v.push_back(ev);
        AMG_HIP(hipEventRecord(ev, s));
        side.push(ev, job);
        su.release_job(job, &deferred);
        Early &e = early[jl];
        e.inv = job.inv;
        e.dA = job.op[0];
        e.dM = job.op[1];
    };
    int j = 0;
    while (true) {
        Level &L = c.lev[j];
        L.n = L.A.n;
        L.dl1inv = c.arena.alloc<double>(L.n);
        const bool last = L.n <= c.o.max_coarse || j + 1 >= c.o.max_levels;
        // exact A_j and M_j solves (the coarsest level included: its A_j is
        // dense in any case, and its mass solves become exact too)
        if (j >= 1 && L.n <= c.o.dense_solve_max) fork_dense(j);
        if (last) break;
        if (!su.coarsen(j)) break;
        ++j;
    }
    c.L = (int)c.lev.size();
    for (auto &L : c.lev) su.level_diag(L);
    // float32 copies for the mixed-precision path
    auto f32 = [&](DCsr &m) {
        if (!m.v || m.nnz == 0) return;
        m.v32 = c.arena.alloc<float>(m.nnz);
        hipLaunchKernelGGL(k_to_f32, dim3(gsz(m.nnz)), dim3(kBlock), 0, s, (long)m.nnz, m.v, m.v32);
    };
    for (auto &L : c.lev) {
        f32(L.A);
        if (L.S.v) {
            f32(L.S);
            f32(L.St);
        }
        if (L.T.v) {
            // S's values on the pattern of T = A S, for the fused coarse
            // correction (after the level loop: off the path to the side stream)
            L.Ts = c.arena.alloc<double>(L.T.nnz);
            hipLaunchKernelGGL(k_align, dim3(gsz((long)(L.n) * kRowLanes)), dim3(kBlock), 0, s, L.n, L.T.rp, L.T.ci, L.S.rp, L.S.ci,
                               L.S.v, L.Ts, c.iscratch + Setup::kFlagAlign);
            f32(L.T);
            L.Ts32 = c.arena.alloc<float>(L.T.nnz);
            hipLaunchKernelGGL(k_to_f32, dim3(gsz(L.T.nnz)), dim3(kBlock), 0, s, (long)L.T.nnz, L.Ts, L.Ts32);
            if (L.T.m <= 65536 && L.T.nnz > 0) {  // T's columns are coarse indices: 16 bits suffice
                L.Tc16 = c.arena.alloc<uint16_t>(L.T.nnz);
                hipLaunchKernelGGL(k_to_u16, dim3(gsz(L.T.nnz)), dim3(kBlock), 0, s, (long)L.T.nnz, L.T.ci, L.Tc16);
            }
        }
        L.dl1inv32 = c.arena.alloc<float>(L.n);
        hipLaunchKernelGGL(k_to_f32, dim3(gsz(L.n)), dim3(kBlock), 0, s, (long)L.n, L.dl1inv, L.dl1inv32);
    }
    // sliced-ELL copies of the finest-level A and M (rows of near-equal length;
    // the prolongator's rows vary too much for the padding to pay)
    su.make_sell(c.lev[0].A);
    su.make_sell(c.lev[0].M);
    su.check_kernels();
    // dense inverse of the coarsest stiffness matrix
    Level &Lc = c.lev[c.L - 1];
    if (Lc.n > c.o.dense_max)
        fail(AMG_ERR_DENSE_TOO_LARGE, "coarsest level has " + std::to_string(Lc.n) + " rows");
    c.nAinv = Lc.n;
    if (early[c.L - 1].inv) {
        c.Ainv = early[c.L - 1].inv;
        c.dAc = early[c.L - 1].dA;
        Lc.Minv = c.Ainv + (size_t)Lc.n * Lc.n;
        Lc.dM = early[c.L - 1].dM;
    } else {
        c.Ainv = su.dense_inverse({&Lc.A});
        c.dAc = su.dense_op(c.Ainv, Lc.n);
    }
    // small coarse levels above the coarsest: exact dense A_j and M_j solves
    for (int j = 1; j + 1 < c.L; ++j) {
        Level &Lv = c.lev[j];
        if (Lv.n > c.o.dense_solve_max) continue;
        Early &e = early[j];
        if (!e.inv || !e.dM.m64) fail(AMG_ERR_HIP, "dense inverse of a small level was not started");
        Lv.Ainv = e.inv;
        Lv.Minv = Lv.Ainv + (size_t)Lv.n * Lv.n;
        Lv.dA = e.dA;
        Lv.dM = e.dM;
    }
    if (!fork_ev.v.empty()) {  // join the side stream
        side.finish();
        AMG_HIP(hipEventRecord(c.side_ev[1], c.side));
        AMG_HIP(hipStreamWaitEvent(s, c.side_ev[1], 0));
        for (void *p : deferred) c.arena.release(p);
    }
    su.check_flags();
}

// Dense practical-form Hessian at level ell-1: H = X^T M_y X + beta M_u,
// X = A^{-1} M_yu, symmetrised and inverted by block Gauss-Jordan sweeps
// (Section 3.2: the coarsest Hessian level is inverted exactly).
void form_dense_hessian(Ctx &c, int ell) {
    Setup su(c);
    hipStream_t s = c.stream;
    su.clear_flags();
    if (ell < 1) ell = 1;
    if (ell > c.L) ell = c.L;
    const int lv = ell - 1;
    Level &L = c.lev[lv];
    const int n = L.n;
    if (c.Hdense) c.arena.release(c.Hdense);
    if (c.Hinv) c.arena.release(c.Hinv);
    if (c.dH.m64) c.arena.release(c.dH.m64);
    if (c.dH.m32) c.arena.release(c.dH.m32);
    c.Hdense = c.Hinv = nullptr;
    c.dH = DenseOp{};
    c.nH = 0;
    c.ell = ell;
    if (n > c.o.dense_max) return;  // solved by loose CG on H (Section 5.2)
    const size_t nn = (size_t)n * n;
    double *Ainv = (lv == c.L - 1) ? c.Ainv : su.dense_inverse({&L.A});
    const uint8_t *mk = lv == 0 ? L.mask : nullptr;
    double *My = c.arena.alloc<double>(nn), *Myu = c.arena.alloc<double>(nn), *Mu = c.arena.alloc<double>(nn);
    for (double *p : {My, Myu, Mu}) su.zero(p, sizeof(double) * nn);
    hipLaunchKernelGGL(k_densify, dim3(gwave(n)), dim3(kBlock), 0, s, n, L.M.rp, L.M.ci, L.M.v, mk, mk, My);
    hipLaunchKernelGGL(k_densify, dim3(gwave(n)), dim3(kBlock), 0, s, n, L.M.rp, L.M.ci, L.M.v, mk,
                       (const uint8_t *)nullptr, Myu);
    hipLaunchKernelGGL(k_densify, dim3(gwave(n)), dim3(kBlock), 0, s, n, L.M.rp, L.M.ci, L.M.v,
                       (const uint8_t *)nullptr, (const uint8_t *)nullptr, Mu);
    double *X = c.arena.alloc<double>(nn), *Y = c.arena.alloc<double>(nn), *XtY = c.arena.alloc<double>(nn);
    const dim3 gg(ceil_div(n, 16), ceil_div(n, 16));
    hipLaunchKernelGGL(k_gemm, gg, dim3(256), 0, s, n, Ainv, 0, Myu, X);
    hipLaunchKernelGGL(k_gemm, gg, dim3(256), 0, s, n, My, 0, X, Y);
    hipLaunchKernelGGL(k_gemm, gg, dim3(256), 0, s, n, X, 1, Y, XtY);
    double *H = c.arena.alloc<double>(nn);
    hipLaunchKernelGGL(k_hsym, dim3(gsz((long)nn)), dim3(kBlock), 0, s, n, XtY, Mu, c.o.beta, H);
    su.check_kernels();
    double *Hf = c.arena.alloc<double>(nn);
    AMG_HIP(hipMemcpyAsync(Hf, H, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    c.Hinv = su.factor_invert(Hf, n);
    c.dH = su.dense_op(c.Hinv, n);
    c.Hdense = H;
    c.nH = n;
    c.ell = ell;
    for (double *p : {My, Myu, Mu, X, Y, XtY}) c.arena.release(p);
    if (Ainv != c.Ainv) c.arena.release(Ainv);
    su.check_flags();
}

}  // namespace amg
