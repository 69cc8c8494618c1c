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
#include <cmath>

#include "ctx.hpp"

#pragma clang fp contract(off)

namespace amg {

namespace {

constexpr int kHS = 2048;        // LDS hash slots per wavefront in the sparse product
constexpr int kMaxRowOut = 1024; // output columns per row at most

__global__ void k_check_sym(int n, const int *rp, const int *ci, const double *v, int *bad) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
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
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double di = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] == i) di = v[p];
        d[i] = di;
        if (!(di > 0.0) && !(mask && mask[i])) atomicAdd(bad, 1);
    }
}

// A_0 = D A D + (I - D): Dirichlet rows and columns leave the pattern, the
// Dirichlet diagonal is one.
__global__ void k_a0_count(int n, const int *rp, const int *ci, const uint8_t *mask, int *cnt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (mask[i]) {
            cnt[i] = 1;
            continue;
        }
        int c = 0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) c += mask[ci[p]] ? 0 : 1;
        cnt[i] = c;
    }
}

__global__ void k_a0_fill(int n, const int *rp, const int *ci, const double *v, const uint8_t *mask,
                          const int *rp0, int *ci0, double *v0) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int o = rp0[i];
        if (mask[i]) {
            ci0[o] = i;
            v0[o] = 1.0;
            continue;
        }
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            if (mask[ci[p]]) continue;
            ci0[o] = ci[p];
            v0[o] = v[p];
            ++o;
        }
    }
}

// exclusive scan, three passes: per-block sums, one-block scan of the sums, add
constexpr int kScanPer = 1024;
__global__ void k_scan_blocks(int n, const int *in, int *bsum) {
    __shared__ int s[kBlock];
    const int base = blockIdx.x * kScanPer;
    int acc = 0;
    for (int k = threadIdx.x; k < kScanPer; k += kBlock) {
        const int i = base + k;
        if (i < n) acc += in[i];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

__global__ void k_scan_sums(int nb, int *bsum, int *total) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int acc = 0;
        for (int b = 0; b < nb; ++b) {
            const int v = bsum[b];
            bsum[b] = acc;
            acc += v;
        }
        *total = acc;
    }
}

__global__ void k_scan_final(int n, const int *in, const int *bsum, int *out, const int *total) {
    __shared__ int s[kScanPer];
    const int base = blockIdx.x * kScanPer;
    for (int k = threadIdx.x; k < kScanPer; k += kBlock) {
        const int i = base + k;
        s[k] = i < n ? in[i] : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = bsum[blockIdx.x];
        for (int k = 0; k < kScanPer; ++k) {
            const int v = s[k];
            s[k] = acc;
            acc += v;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kScanPer; k += kBlock) {
        const int i = base + k;
        if (i < n) out[i] = s[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *total;
}

__global__ void k_l1(int n, const int *rp, const double *v, double *dl1inv, double *dl1) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) s = s + fabs(v[p]);
        dl1[i] = s;
        dl1inv[i] = 1.0 / s;
    }
}

__global__ void k_inv(int n, const double *d, double *dinv) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dinv[i] = 1.0 / d[i];
}

__global__ void k_strength(int n, const int *rp, const int *ci, const double *v, const double *d,
                           const uint8_t *mask, double t, uint8_t *flag, int *cnt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int c = 0;
        const bool mi = mask && mask[i];
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int k = ci[p];
            bool s = false;
            if (k != i && !mi && !(mask && mask[k])) {
                const double a = v[p];
                const double lhs = a * a;
                const double dd = d[i] * d[k];
                const double rhs = t * dd;
                s = lhs >= rhs;
            }
            flag[p] = s;
            c += s;
        }
        cnt[i] = c;
    }
}

__global__ void k_strong_fill(int n, const int *rp, const int *ci, const double *v, const uint8_t *flag,
                              const int *srp, int *sci, double *sabs) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int o = srp[i];
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            if (flag[p]) {
                sci[o] = ci[p];
                sabs[o] = fabs(v[p]);
                ++o;
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

__global__ void k_mis_m1(int n, const int *srp, const int *sci, const uint64_t *h, const int8_t *st,
                         int *m1) {
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
                         int8_t *st) {
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

__global__ void k_mis_r1(int n, const int *srp, const int *sci, const int8_t *st, uint8_t *r1) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint8_t any = st[i] == ROOT;
        for (int p = srp[i]; p < srp[i + 1] && !any; ++p) any = st[sci[p]] == ROOT;
        r1[i] = any;
    }
}

__global__ void k_mis_r2(int n, const int *srp, const int *sci, const uint8_t *r1, int8_t *st, int *undec) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (st[i] != UNDEC) continue;
        bool any = r1[i];
        for (int p = srp[i]; p < srp[i + 1] && !any; ++p) any = r1[sci[p]];
        if (any) st[i] = OUT;
        else atomicAdd(undec, 1);
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
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (mask && mask[i]) continue;
        const double r = dl1[i] / d[i];
        atomicMax(maxbits, (unsigned long long)__double_as_longlong(r));  // r > 0: bit order = value order
    }
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
__global__ void k_smooth(int n, const int *rp, const int *ci, double *v, const int *agg, const double *d,
                         double omega) {
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

// rows of the transpose: rank sort by column index, one wavefront per row
// (the keys of a row are distinct row indices of the source matrix)
__global__ __launch_bounds__(kBlock) void k_row_sort(int m, const int *rp, const int *ci_in, const double *v_in,
                                                     int *ci_out, double *v_out) {
    const int lane = threadIdx.x % 64;
    const int w = (blockIdx.x * kBlock + threadIdx.x) / 64;
    const int nw = gridDim.x * kBlock / 64;
    for (int r = w; r < m; r += nw) {
        const int s = rp[r], e = rp[r + 1];
        for (int a = s + lane; a < e; a += 64) {
            const int key = ci_in[a];
            int rank = 0;
            for (int b = s; b < e; ++b) rank += ci_in[b] < key;
            ci_out[s + rank] = key;
            v_out[s + rank] = v_in[a];
        }
    }
}

// ---- sparse product C = A B, one wavefront per row of A, LDS hash of the
// output columns; values summed over the stored A[i,k] in ascending k ----
__device__ __forceinline__ int hash_insert(int *tab, int key, int *ucount, int *ovf) {
    unsigned h = ((unsigned)key * 2654435761u) & (kHS - 1);
    for (int probe = 0; probe < kHS; ++probe) {
        const int old = atomicCAS(&tab[h], -1, key);
        if (old == -1) {
            atomicAdd(ucount, 1);
            return 1;
        }
        if (old == key) return 0;
        h = (h + 1) & (kHS - 1);
    }
    atomicOr(ovf, 1);
    return 0;
}

__global__ __launch_bounds__(kBlock) void k_spgemm_count(int n, const int *arp, const int *aci,
                                                         const int *brp, const int *bci, int *cnt,
                                                         int *ovf) {
    __shared__ int tab[4][kHS];
    __shared__ int uc[4];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int base = blockIdx.x * 4; base < n; base += gridDim.x * 4) {
        const int row = base + w;
        for (int s = lane; s < kHS; s += 64) tab[w][s] = -1;
        if (lane == 0) uc[w] = 0;
        __syncthreads();
        if (row < n) {
            for (int p = arp[row] + lane; p < arp[row + 1]; p += 64) {
                const int k = aci[p];
                for (int q = brp[k]; q < brp[k + 1]; ++q) hash_insert(tab[w], bci[q], &uc[w], ovf);
            }
        }
        __syncthreads();
        if (row < n && lane == 0) {
            cnt[row] = uc[w];
            if (uc[w] > kMaxRowOut) atomicOr(ovf, 1);
        }
        __syncthreads();
    }
}

// Fill variant for short rows of B: one lane per output column, summing the
// products over the stored A[i,k] in ascending k (binary search in row k of B).
__global__ __launch_bounds__(kBlock) void k_spgemm_fill_search(int n, const int *arp, const int *aci,
                                                               const double *av, const int *brp,
                                                               const int *bci, const double *bv,
                                                               const int *crp, int *cci, double *cv,
                                                               int *ovf) {
    __shared__ int tab[4][kHS];
    __shared__ int lst[4][kMaxRowOut];
    __shared__ int srt[4][kMaxRowOut];
    __shared__ int uc[4], uc2[4];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int base = blockIdx.x * 4; base < n; base += gridDim.x * 4) {
        const int row = base + w;
        for (int s = lane; s < kHS; s += 64) tab[w][s] = -1;
        if (lane == 0) {
            uc[w] = 0;
            uc2[w] = 0;
        }
        __syncthreads();
        if (row < n) {
            for (int p = arp[row] + lane; p < arp[row + 1]; p += 64) {
                const int k = aci[p];
                for (int q = brp[k]; q < brp[k + 1]; ++q) hash_insert(tab[w], bci[q], &uc[w], ovf);
            }
        }
        __syncthreads();
        const int u = row < n ? uc[w] : 0;
        const bool ok = u <= kMaxRowOut;
        if (row < n && ok) {
            for (int s = lane; s < kHS; s += 64) {
                const int key = tab[w][s];
                if (key >= 0) lst[w][atomicAdd(&uc2[w], 1)] = key;
            }
        }
        __syncthreads();
        if (row < n && ok) {
            for (int e = lane; e < u; e += 64) {
                const int key = lst[w][e];
                int rank = 0;
                for (int f = 0; f < u; ++f) rank += lst[w][f] < key;
                srt[w][rank] = key;
            }
        }
        __syncthreads();
        if (row < n && ok) {
            const int cs = crp[row];
            const int a0 = arp[row], a1 = arp[row + 1];
            for (int e = lane; e < u; e += 64) {
                const int J = srt[w][e];
                double acc = 0.0;
                for (int p = a0; p < a1; ++p) {
                    const int k = aci[p];
                    int lo = brp[k], hi = brp[k + 1] - 1;
                    while (lo <= hi) {
                        const int mid = (lo + hi) >> 1;
                        const int cm = bci[mid];
                        if (cm == J) {
                            const double prod = av[p] * bv[mid];
                            acc = acc + prod;
                            break;
                        }
                        if (cm < J) lo = mid + 1;
                        else hi = mid - 1;
                    }
                }
                cci[cs + e] = J;
                cv[cs + e] = acc;
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int hash_find(const int *tab, int key) {
    unsigned h = ((unsigned)key * 2654435761u) & (kHS - 1);
    for (int probe = 0; probe < kHS; ++probe) {
        const int v = tab[h];
        if (v == key || v == -1) return v == key ? (int)h : -1;
        h = (h + 1) & (kHS - 1);
    }
    return -1;
}

// Fill: rebuild the row's hash of output columns, give every column its rank
// in ascending order (the output position), then accumulate the products in
// LDS walking the stored A[i,k] in ascending k; for one k the lanes share out
// the row of B, whose columns are distinct, so every output entry receives its
// products strictly in ascending k: the same rounded sums as a sequential loop.
constexpr int kFillWaves = 2;
__global__ __launch_bounds__(64 * kFillWaves) void k_spgemm_fill(int n, const int *arp, const int *aci,
                                                                const double *av, const int *brp,
                                                                const int *bci, const double *bv,
                                                                const int *crp, int *cci, double *cv,
                                                                int *ovf) {
    __shared__ int tab[kFillWaves][kHS];
    __shared__ int pos[kFillWaves][kHS];
    __shared__ int lst[kFillWaves][kMaxRowOut];
    __shared__ double acc[kFillWaves][kMaxRowOut];
    __shared__ int uc[kFillWaves], uc2[kFillWaves];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int base = blockIdx.x * kFillWaves; base < n; base += gridDim.x * kFillWaves) {
        const int row = base + w;
        for (int s = lane; s < kHS; s += 64) tab[w][s] = -1;
        if (lane == 0) {
            uc[w] = 0;
            uc2[w] = 0;
        }
        __syncthreads();
        if (row < n) {
            for (int p = arp[row] + lane; p < arp[row + 1]; p += 64) {
                const int k = aci[p];
                for (int q = brp[k]; q < brp[k + 1]; ++q) hash_insert(tab[w], bci[q], &uc[w], ovf);
            }
        }
        __syncthreads();
        const int u = row < n ? uc[w] : 0;
        const bool ok = row < n && u <= kMaxRowOut;
        if (ok) {
            for (int s = lane; s < kHS; s += 64) {
                const int key = tab[w][s];
                if (key >= 0) lst[w][atomicAdd(&uc2[w], 1)] = key;
            }
        }
        __syncthreads();
        if (ok) {
            const int cs = crp[row];
            for (int s = lane; s < kHS; s += 64) {
                const int key = tab[w][s];
                if (key < 0) continue;
                int rank = 0;
                for (int f = 0; f < u; ++f) rank += lst[w][f] < key;
                pos[w][s] = rank;
                cci[cs + rank] = key;
                acc[w][rank] = 0.0;
            }
        }
        __syncthreads();
        if (ok) {
            const int a0 = arp[row], a1 = arp[row + 1];
            for (int p = a0; p < a1; ++p) {
                const int k = aci[p];
                const double a = av[p];
                for (int q = brp[k] + lane; q < brp[k + 1]; q += 64) {
                    const int slot = hash_find(tab[w], bci[q]);
                    if (slot < 0) {  // cannot happen: every key was inserted above
                        atomicOr(ovf, 2);
                        continue;
                    }
                    const int r = pos[w][slot];
                    const double prod = a * bv[q];
                    acc[w][r] = acc[w][r] + prod;
                }
            }
        }
        __syncthreads();
        if (ok) {
            const int cs = crp[row];
            for (int e = lane; e < u; e += 64) cv[cs + e] = acc[w][e];
        }
        __syncthreads();
    }
}

// lower triangle := upper triangle (symbolically symmetric pattern)
__global__ void k_mirror(int n, const int *rp, const int *ci, double *v, int *bad) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
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

// ---- dense kernels (coarsest level) ----
__global__ void k_densify(int n, const int *rp, const int *ci, const double *v, const uint8_t *rmask,
                          const uint8_t *cmask, double *D) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const bool rk = !(rmask && rmask[i]);
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int k = ci[p];
            const bool ck = !(cmask && cmask[k]);
            D[(size_t)i * n + k] = (rk && ck) ? v[p] : 0.0;
        }
    }
}

// Tiled right-looking Cholesky of the lower triangle (tiles of kTB): per tile
// column kb, factor the diagonal tile in LDS, solve the panel below it, then
// update the trailing lower tiles.  Only the lower triangle is read later.
constexpr int kTB = 32;

__global__ __launch_bounds__(kBlock) void k_potrf_tile(int n, double *D, int k0, int *bad) {
    __shared__ double T[kTB][kTB + 1];
    __shared__ double piv;
    const int tb = min(kTB, n - k0);
    const int t = threadIdx.x;
    for (int e = t; e < tb * tb; e += kBlock) T[e / tb][e % tb] = D[(size_t)(k0 + e / tb) * n + k0 + e % tb];
    __syncthreads();
    for (int k = 0; k < tb; ++k) {
        if (t == 0) {
            const double a = T[k][k];
            if (!(a > 0.0)) {
                atomicOr(bad, 1);
                piv = 1.0;
            } else {
                piv = sqrt(a);
            }
            T[k][k] = piv;
        }
        __syncthreads();
        if (t > k && t < tb) T[t][k] /= piv;
        __syncthreads();
        for (int e = t; e < tb * tb; e += kBlock) {
            const int i = e / tb, j = e % tb;
            if (j > k && j <= i) T[i][j] -= T[i][k] * T[j][k];
        }
        __syncthreads();
    }
    for (int e = t; e < tb * tb; e += kBlock) {
        const int i = e / tb, j = e % tb;
        if (j <= i) D[(size_t)(k0 + i) * n + k0 + j] = T[i][j];
    }
}

// panel: rows below the diagonal tile, X = A_ik L_kk^{-T}, one wavefront per row tile
__global__ __launch_bounds__(64) void k_trsm_tile(int n, double *D, int k0) {
    __shared__ double Lk[kTB][kTB + 1];
    const int tb = min(kTB, n - k0);
    const int t = threadIdx.x;
    for (int e = t; e < tb * tb; e += 64) Lk[e / tb][e % tb] = D[(size_t)(k0 + e / tb) * n + k0 + e % tb];
    __syncthreads();
    const int r = k0 + tb + blockIdx.x * kTB + t;
    if (t >= kTB || r >= n) return;
    double x[kTB];
#pragma unroll
    for (int j = 0; j < kTB; ++j) x[j] = j < tb ? D[(size_t)r * n + k0 + j] : 0.0;
#pragma unroll
    for (int j = 0; j < kTB; ++j) {
        if (j < tb) {
            double v = x[j];
            for (int m = 0; m < j; ++m) v -= x[m] * Lk[j][m];
            x[j] = v / Lk[j][j];
        }
    }
#pragma unroll
    for (int j = 0; j < kTB; ++j)
        if (j < tb) D[(size_t)r * n + k0 + j] = x[j];
}

// trailing update A_ij -= L_ik L_jk^T for tile pairs i >= j after tile column k0
__global__ __launch_bounds__(kBlock) void k_syrk_tile(int n, double *D, int k0) {
    __shared__ double Li[kTB][kTB + 1], Lj[kTB][kTB + 1];
    const int tb = min(kTB, n - k0);
    const int s0 = k0 + tb;  // first trailing row
    const long p = blockIdx.x;
    long ti = (long)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > p) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= p) ++ti;
    const long tj = p - ti * (ti + 1) / 2;
    const int r0 = s0 + (int)ti * kTB, c0 = s0 + (int)tj * kTB;
    const int t = threadIdx.x;
    for (int e = t; e < kTB * kTB; e += kBlock) {
        const int a = e / kTB, m = e % kTB;
        Li[a][m] = (r0 + a < n && m < tb) ? D[(size_t)(r0 + a) * n + k0 + m] : 0.0;
        Lj[a][m] = (c0 + a < n && m < tb) ? D[(size_t)(c0 + a) * n + k0 + m] : 0.0;
    }
    __syncthreads();
    for (int e = t; e < kTB * kTB; e += kBlock) {
        const int a = e / kTB, b = e % kTB;
        const int i = r0 + a, j = c0 + b;
        if (i >= n || j >= n || j > i) continue;
        double acc = 0.0;
        for (int m = 0; m < tb; ++m) acc += Li[a][m] * Lj[b][m];
        D[(size_t)i * n + j] -= acc;
    }
}

// Lt = L^T for the lower triangle (column k of L becomes a contiguous row)
__global__ void k_lower_transpose(int n, const double *L, double *Lt) {
    const long tot = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        if (j <= i) Lt[(size_t)j * n + i] = L[e];
    }
}

// Inverse from the Cholesky factor: R columns of the identity per workgroup,
// forward solve L y = e_j reading rows of L^T, backward solve L^T x = y
// reading rows of L (both contiguous), vectors in LDS, one barrier per step.
// Thread t owns the entries i = t (mod blockDim); the row needed at the next
// step is loaded before the current step's updates so its latency overlaps.
constexpr int kInvP = 16;  // entries per thread: n <= kInvP * kBlock = 4096
__global__ __launch_bounds__(kBlock) void k_chol_inv(int n, int R, const double *Lf, const double *Lt,
                                                     double *inv) {
    extern __shared__ double sm[];
    double *y = sm;          // [R][n]
    double *w = sm + R * n;  // [R][n]: finished entries
    const int j0 = blockIdx.x * R;
    const int t = threadIdx.x, B = blockDim.x;
    for (int e = t; e < R * n; e += B) {
        const int q = e / n, i = e % n;
        y[e] = (j0 + q < n && i == j0 + q) ? 1.0 : 0.0;
    }
    double cur[kInvP], nxt[kInvP];
#pragma unroll
    for (int m = 0; m < kInvP; ++m) {
        const int i = t + m * B;
        cur[m] = i < n ? Lt[i] : 0.0;  // row 0 of L^T
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (k + 1 < n) {
            const double *nr = Lt + (size_t)(k + 1) * n;
#pragma unroll
            for (int m = 0; m < kInvP; ++m) {
                const int i = t + m * B;
                nxt[m] = i < n ? nr[i] : 0.0;
            }
        }
        const double dk = Lf[(size_t)k * n + k];
        for (int q = 0; q < R; ++q) {
            const double yk = y[q * n + k] / dk;
#pragma unroll
            for (int m = 0; m < kInvP; ++m) {
                const int i = t + m * B;
                if (i > k && i < n) y[q * n + i] -= cur[m] * yk;
            }
            if (t == 0) w[q * n + k] = yk;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kInvP; ++m) cur[m] = nxt[m];
    }
#pragma unroll
    for (int m = 0; m < kInvP; ++m) {
        const int i = t + m * B;
        cur[m] = i < n ? Lf[(size_t)(n - 1) * n + i] : 0.0;
    }
    for (int k = n - 1; k >= 0; --k) {
        if (k > 0) {
            const double *pr = Lf + (size_t)(k - 1) * n;
#pragma unroll
            for (int m = 0; m < kInvP; ++m) {
                const int i = t + m * B;
                nxt[m] = i < n ? pr[i] : 0.0;
            }
        }
        const double dk = Lf[(size_t)k * n + k];
        for (int q = 0; q < R; ++q) {
            const double xk = w[q * n + k] / dk;
#pragma unroll
            for (int m = 0; m < kInvP; ++m) {
                const int i = t + m * B;
                if (i < k) w[q * n + i] -= cur[m] * xk;
            }
            if (t == 0) y[q * n + k] = xk;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kInvP; ++m) cur[m] = nxt[m];
    }
    for (int e = t; e < R * n; e += B) {
        const int q = e / n, i = e % n;
        if (j0 + q < n) inv[(size_t)(j0 + q) * n + i] = y[e];
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

struct Setup {
    Ctx &c;
    hipStream_t s;
    explicit Setup(Ctx &cc) : c(cc), s(cc.stream) {}

    int read_int(const int *d) {
        AMG_HIP(hipMemcpyAsync(c.hiscr, d, sizeof(int), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        return c.hiscr[0];
    }

    void zero(void *p, size_t bytes) { AMG_HIP(hipMemsetAsync(p, 0, bytes, s)); }

    // out[0..n] exclusive scan of cnt[0..n-1]; returns the total
    int scan(const int *cnt, int *out, int n) {
        const int nb = std::max(1, ceil_div(n, kScanPer));
        int *bsum = c.arena.alloc<int>(nb);
        hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kBlock), 0, s, n, cnt, bsum);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(64), 0, s, nb, bsum, c.iscratch + 8);
        hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kBlock), 0, s, n, cnt, bsum, out, c.iscratch + 8);
        const int total = read_int(c.iscratch + 8);
        c.arena.release(bsum);
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
        hipLaunchKernelGGL(k_check_sym, dim3(gsz(d.n)), dim3(kBlock), 0, s, d.n, d.rp, d.ci, d.v, c.iscratch);
        check_kernels();
        AMG_HIP(hipMemcpyAsync(c.hiscr, c.iscratch, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        if (c.hiscr[1]) fail(AMG_ERR_ARG, std::string(name) + ": columns not sorted/unique within a row");
        if (c.hiscr[0]) fail(AMG_ERR_NOT_SYMMETRIC, std::string(name) + " is not exactly symmetric");
    }

    DCsr spgemm(const DCsr &A, const DCsr &B) {
        DCsr C;
        C.n = A.n;
        C.m = B.m;
        int *cnt = c.arena.alloc<int>(A.n + 1);
        C.rp = c.arena.alloc<int>(A.n + 1);
        zero(c.iscratch + 4, sizeof(int));
        const int g = std::min(4096, std::max(1, ceil_div(A.n, 4)));
        hipLaunchKernelGGL(k_spgemm_count, dim3(g), dim3(kBlock), 0, s, A.n, A.rp, A.ci, B.rp, B.ci, cnt,
                           c.iscratch + 4);
        check_kernels();
        if (read_int(c.iscratch + 4))
            fail(AMG_ERR_CAPACITY, "sparse product row exceeds " + std::to_string(kMaxRowOut) + " columns");
        C.nnz = scan(cnt, C.rp, A.n);
        C.ci = c.arena.alloc<int>(C.nnz);
        C.v = c.arena.alloc<double>(C.nnz);
        if ((double)B.nnz <= 8.0 * (double)B.n) {  // short rows of B: per-column search
            hipLaunchKernelGGL(k_spgemm_fill_search, dim3(g), dim3(kBlock), 0, s, A.n, A.rp, A.ci, A.v, B.rp, B.ci,
                               B.v, C.rp, C.ci, C.v, c.iscratch + 4);
        } else {
            const int gf = std::min(8192, std::max(1, ceil_div(A.n, kFillWaves)));
            hipLaunchKernelGGL(k_spgemm_fill, dim3(gf), dim3(64 * kFillWaves), 0, s, A.n, A.rp, A.ci, A.v, B.rp,
                               B.ci, B.v, C.rp, C.ci, C.v, c.iscratch + 4);
        }
        check_kernels();
        c.arena.release(cnt);
        return C;
    }

    DCsr transpose(const DCsr &A) {
        DCsr T;
        T.n = A.m;
        T.m = A.n;
        T.nnz = A.nnz;
        int *cnt = c.arena.alloc<int>(T.n + 1);
        int *fill = c.arena.alloc<int>(T.n + 1);
        zero(cnt, sizeof(int) * (T.n + 1));
        zero(fill, sizeof(int) * (T.n + 1));
        T.rp = c.arena.alloc<int>(T.n + 1);
        T.ci = c.arena.alloc<int>(T.nnz);
        T.v = c.arena.alloc<double>(T.nnz);
        int *tci = c.arena.alloc<int>(T.nnz);
        double *tv = c.arena.alloc<double>(T.nnz);
        hipLaunchKernelGGL(k_t_count, dim3(gsz(A.n)), dim3(kBlock), 0, s, A.n, A.rp, A.ci, cnt);
        scan(cnt, T.rp, T.n);
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

    DCsr galerkin(const DCsr &S, const DCsr &St, const DCsr &A) {
        DCsr T = spgemm(A, S);
        DCsr C = spgemm(St, T);
        zero(c.iscratch + 5, sizeof(int));
        hipLaunchKernelGGL(k_mirror, dim3(gsz(C.n)), dim3(kBlock), 0, s, C.n, C.rp, C.ci, C.v, c.iscratch + 5);
        check_kernels();
        if (read_int(c.iscratch + 5)) fail(AMG_ERR_ARG, "coarse matrix pattern is not symmetric");
        c.arena.release(T.rp);
        c.arena.release(T.ci);
        c.arena.release(T.v);
        return C;
    }

    // returns false when coarsening stops at level j
    bool coarsen(int j) {
        Level &L0 = c.lev[j];
        const DCsr &A = L0.A;
        const int n = A.n;
        const uint8_t *mask = L0.mask;
        double *d = c.arena.alloc<double>(n);
        zero(c.iscratch, sizeof(int));
        hipLaunchKernelGGL(k_diag, dim3(gsz(n)), dim3(kBlock), 0, s, n, A.rp, A.ci, A.v, mask, d, c.iscratch);
        if (read_int(c.iscratch)) fail(AMG_ERR_NOT_SPD, "non-positive diagonal at level " + std::to_string(j));
        // strength graph
        const double theta = c.o.theta0 * std::ldexp(1.0, -j);
        const double t = theta * theta;
        uint8_t *flag = c.arena.alloc<uint8_t>(A.nnz);
        int *cnt = c.arena.alloc<int>(n + 1);
        int *srp = c.arena.alloc<int>(n + 1);
        hipLaunchKernelGGL(k_strength, dim3(gsz(n)), dim3(kBlock), 0, s, n, A.rp, A.ci, A.v, d, mask, t, flag,
                           cnt);
        const int snnz = scan(cnt, srp, n);
        int *sci = c.arena.alloc<int>(snnz);
        double *sabs = c.arena.alloc<double>(snnz);
        hipLaunchKernelGGL(k_strong_fill, dim3(gsz(n)), dim3(kBlock), 0, s, n, A.rp, A.ci, A.v, flag, srp, sci,
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
        for (int round = 0;; ++round) {
            if (round > n + 1) fail(AMG_ERR_ARG, "independent-set rounds did not terminate");
            hipLaunchKernelGGL(k_mis_m1, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, h, st, m1);
            hipLaunchKernelGGL(k_mis_m2, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, h, m1, st);
            hipLaunchKernelGGL(k_mis_r1, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, st, r1);
            zero(c.iscratch + 6, sizeof(int));
            hipLaunchKernelGGL(k_mis_r2, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, r1, st, c.iscratch + 6);
            check_kernels();
            if (read_int(c.iscratch + 6) == 0) break;
        }
        L0.root = c.arena.alloc<uint8_t>(n);
        int *cid = c.arena.alloc<int>(n + 1);
        hipLaunchKernelGGL(k_root_flags, dim3(gsz(n)), dim3(kBlock), 0, s, n, st, L0.root, cnt);
        const int nc = scan(cnt, cid, n);
        L0.agg = c.arena.alloc<int>(n);
        uint8_t *p2 = c.arena.alloc<uint8_t>(n);
        hipLaunchKernelGGL(k_phase2, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, sabs, L0.root, cid, mask,
                           L0.agg, p2);
        zero(c.iscratch + 7, sizeof(int));
        hipLaunchKernelGGL(k_phase3, dim3(gsz(n)), dim3(kBlock), 0, s, n, srp, sci, sabs, p2, L0.agg,
                           c.iscratch + 7);
        check_kernels();
        if (read_int(c.iscratch + 7)) fail(AMG_ERR_ARG, "aggregation left a node unassigned");
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
        hipLaunchKernelGGL(k_l1, dim3(gsz(n)), dim3(kBlock), 0, s, n, A.rp, A.v, L0.dl1inv, dl1);
        unsigned long long *mb = reinterpret_cast<unsigned long long *>(c.dscratch);
        zero(mb, sizeof(unsigned long long));
        hipLaunchKernelGGL(k_rho, dim3(gsz(n)), dim3(kBlock), 0, s, n, dl1, d, mask, mb);
        check_kernels();
        AMG_HIP(hipMemcpyAsync(c.hscr, c.dscratch, sizeof(double), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        L0.rho = c.hscr[0];
        L0.omega = (4.0 / 3.0) / L0.rho;
        c.arena.release(dl1);
        // tentative prolongator, then S = (I - omega D^{-1} A) P_tent
        DCsr P;
        P.n = n;
        P.m = nc;
        P.rp = c.arena.alloc<int>(n + 1);
        hipLaunchKernelGGL(k_ptent_count, dim3(gsz(n)), dim3(kBlock), 0, s, n, L0.agg, cnt);
        P.nnz = scan(cnt, P.rp, n);
        P.ci = c.arena.alloc<int>(P.nnz);
        P.v = c.arena.alloc<double>(P.nnz);
        hipLaunchKernelGGL(k_ptent_fill, dim3(gsz(n)), dim3(kBlock), 0, s, n, L0.agg, P.rp, P.ci, P.v);
        DCsr S = spgemm(A, P);
        hipLaunchKernelGGL(k_smooth, dim3(gsz(n)), dim3(kBlock), 0, s, n, S.rp, S.ci, S.v, L0.agg, d, L0.omega);
        check_kernels();
        for (void *p : {(void *)P.rp, (void *)P.ci, (void *)P.v, (void *)cnt, (void *)d}) c.arena.release(p);
        L0.S = S;
        L0.St = transpose(S);
        Level nx;
        nx.n = nc;
        nx.A = galerkin(L0.S, L0.St, A);
        nx.M = galerkin(L0.S, L0.St, L0.M);
        c.lev.push_back(nx);
        return true;
    }

    void level_diag(Level &L) {
        const int n = L.A.n;
        L.n = n;
        if (!L.dl1inv) L.dl1inv = c.arena.alloc<double>(n);
        double *dl1 = c.arena.alloc<double>(n);
        hipLaunchKernelGGL(k_l1, dim3(gsz(n)), dim3(kBlock), 0, s, n, L.A.rp, L.A.v, L.dl1inv, dl1);
        double *md = c.arena.alloc<double>(n);
        L.mdinv = c.arena.alloc<double>(n);
        zero(c.iscratch, sizeof(int));
        hipLaunchKernelGGL(k_diag, dim3(gsz(n)), dim3(kBlock), 0, s, n, L.M.rp, L.M.ci, L.M.v,
                           (const uint8_t *)nullptr, md, c.iscratch);
        hipLaunchKernelGGL(k_inv, dim3(gsz(n)), dim3(kBlock), 0, s, n, md, L.mdinv);
        check_kernels();
        if (read_int(c.iscratch)) fail(AMG_ERR_NOT_SPD, "mass matrix has a non-positive diagonal");
        c.arena.release(dl1);
        c.arena.release(md);
    }

    // dense inverse of a (masked) sparse SPD matrix through its Cholesky factor
    double *dense_inverse(const DCsr &A, const uint8_t *mask, bool unit_masked_diag) {
        const int n = A.n;
        double *D = c.arena.alloc<double>((size_t)n * n);
        zero(D, sizeof(double) * n * n);
        hipLaunchKernelGGL(k_densify, dim3(gsz(n)), dim3(kBlock), 0, s, n, A.rp, A.ci, A.v,
                           (const uint8_t *)nullptr, (const uint8_t *)nullptr, D);
        (void)mask;
        (void)unit_masked_diag;
        return factor_invert(D, n);
    }

    double *factor_invert(double *D, int n) {
        zero(c.iscratch + 9, sizeof(int));
        for (int k0 = 0; k0 < n; k0 += kTB) {
            hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(kBlock), 0, s, n, D, k0, c.iscratch + 9);
            const int rest = n - (k0 + kTB);
            if (rest <= 0) break;
            const int tiles = ceil_div(rest, kTB);
            hipLaunchKernelGGL(k_trsm_tile, dim3(tiles), dim3(64), 0, s, n, D, k0);
            hipLaunchKernelGGL(k_syrk_tile, dim3(tiles * (tiles + 1) / 2), dim3(kBlock), 0, s, n, D, k0);
        }
        check_kernels();
        if (read_int(c.iscratch + 9)) fail(AMG_ERR_NOT_SPD, "dense Cholesky met a non-positive pivot");
        double *inv = c.arena.alloc<double>((size_t)n * n);
        double *Lt = c.arena.alloc<double>((size_t)n * n);
        hipLaunchKernelGGL(k_lower_transpose, dim3(gsz((long)n * n)), dim3(kBlock), 0, s, n, D, Lt);
        // LDS: 2 R n doubles within 64 KiB (n <= 4096)
        const int R = std::max(1, std::min(8, 4096 / n));
        hipLaunchKernelGGL(k_chol_inv, dim3(ceil_div(n, R)), dim3(kBlock), sizeof(double) * 2 * R * n, s, n, R, D,
                           Lt, inv);
        check_kernels();
        c.arena.release(D);
        c.arena.release(Lt);
        return inv;
    }
};

}  // namespace

void build_hierarchy(Ctx &c, const amg_csr &Ain, const amg_csr &Min, const uint8_t *dirichlet) {
    Setup su(c);
    hipStream_t s = c.stream;
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
        DCsr A0;
        A0.n = A0.m = N;
        int *cnt = c.arena.alloc<int>(N + 1);
        A0.rp = c.arena.alloc<int>(N + 1);
        hipLaunchKernelGGL(k_a0_count, dim3(gsz(N)), dim3(kBlock), 0, s, N, A.rp, A.ci, c.mask0, cnt);
        A0.nnz = su.scan(cnt, A0.rp, N);
        A0.ci = c.arena.alloc<int>(A0.nnz);
        A0.v = c.arena.alloc<double>(A0.nnz);
        hipLaunchKernelGGL(k_a0_fill, dim3(gsz(N)), dim3(kBlock), 0, s, N, A.rp, A.ci, A.v, c.mask0, A0.rp,
                           A0.ci, A0.v);
        su.check_kernels();
        c.arena.release(cnt);
        c.arena.release(A.rp);
        c.arena.release(A.ci);
        c.arena.release(A.v);
        l0.A = A0;
    } else {
        l0.A = A;
    }
    c.lev.clear();
    c.lev.push_back(l0);
    int j = 0;
    while (true) {
        Level &L = c.lev[j];
        L.n = L.A.n;
        L.dl1inv = c.arena.alloc<double>(L.n);
        if (L.n <= c.o.max_coarse || j + 1 >= c.o.max_levels) break;
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
        L.dl1inv32 = c.arena.alloc<float>(L.n);
        hipLaunchKernelGGL(k_to_f32, dim3(gsz(L.n)), dim3(kBlock), 0, s, (long)L.n, L.dl1inv, L.dl1inv32);
    }
    su.check_kernels();
    // dense inverse of the coarsest stiffness matrix
    Level &Lc = c.lev[c.L - 1];
    if (Lc.n > c.o.dense_max)
        fail(AMG_ERR_DENSE_TOO_LARGE, "coarsest level has " + std::to_string(Lc.n) + " rows");
    c.nAinv = Lc.n;
    c.Ainv = su.dense_inverse(Lc.A, nullptr, false);
    // small coarse levels above the coarsest: exact dense A_j and M_j solves
    for (int j = 1; j + 1 < c.L; ++j) {
        Level &Lv = c.lev[j];
        if (Lv.n > c.o.dense_solve_max) continue;
        Lv.Ainv = su.dense_inverse(Lv.A, nullptr, false);
        Lv.Minv = su.dense_inverse(Lv.M, nullptr, false);
    }
    AMG_HIP(hipStreamSynchronize(s));
}

// Dense practical-form Hessian at level ell-1: H = X^T M_y X + beta M_u,
// X = A^{-1} M_yu, symmetrised and inverted through its Cholesky factor
// (Section 3.2: the coarsest Hessian level is inverted exactly).
void form_dense_hessian(Ctx &c, int ell) {
    Setup su(c);
    hipStream_t s = c.stream;
    if (ell < 1) ell = 1;
    if (ell > c.L) ell = c.L;
    const int lv = ell - 1;
    Level &L = c.lev[lv];
    const int n = L.n;
    if (c.Hdense) c.arena.release(c.Hdense);
    if (c.Hinv) c.arena.release(c.Hinv);
    c.Hdense = c.Hinv = nullptr;
    c.nH = 0;
    c.ell = ell;
    if (n > c.o.dense_max) return;  // solved by loose CG on H (Section 5.2)
    const size_t nn = (size_t)n * n;
    double *Ainv = (lv == c.L - 1) ? c.Ainv : su.dense_inverse(L.A, nullptr, false);
    const uint8_t *mk = lv == 0 ? L.mask : nullptr;
    double *My = c.arena.alloc<double>(nn), *Myu = c.arena.alloc<double>(nn), *Mu = c.arena.alloc<double>(nn);
    for (double *p : {My, Myu, Mu}) su.zero(p, sizeof(double) * nn);
    hipLaunchKernelGGL(k_densify, dim3(gsz(n)), dim3(kBlock), 0, s, n, L.M.rp, L.M.ci, L.M.v, mk, mk, My);
    hipLaunchKernelGGL(k_densify, dim3(gsz(n)), dim3(kBlock), 0, s, n, L.M.rp, L.M.ci, L.M.v, mk,
                       (const uint8_t *)nullptr, Myu);
    hipLaunchKernelGGL(k_densify, dim3(gsz(n)), dim3(kBlock), 0, s, n, L.M.rp, L.M.ci, L.M.v,
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
    c.Hdense = H;
    c.nH = n;
    c.ell = ell;
    for (double *p : {My, Myu, Mu, X, Y, XtY}) c.arena.release(p);
    if (Ainv != c.Ainv) c.arena.release(Ainv);
    AMG_HIP(hipStreamSynchronize(s));
}

}  // namespace amg
