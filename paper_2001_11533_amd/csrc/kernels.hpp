// Solve-phase device code for gfx950: row-blocked CSR SpMV/SpMM with fused
// epilogues, elementwise kernels with fused dot products, deterministic
// two-stage grid reductions, and the dense coarse-level apply.
//
// Layout: every work vector is row-major [n x NB] (entry (i, c) at i*NB + c),
// NB in {1, 2, 4, 8, 16}.  A row of a CSR matrix is handled by LPR =
// max(8, NB) consecutive lanes of one wavefront: lane l works on column
// c = l % NB and on the stored entries g, g + G, ... of the row, g = l / NB,
// G = LPR / NB; the G partial sums are combined with wavefront shuffles.
// For NB >= 8 every lane owns one column and the NB lanes of a row read the
// same (col, val) entry, so the matrix is fetched once per row for all
// right-hand sides while the x gathers are NB-contiguous.
//
// Reductions are deterministic: each workgroup reduces its contribution in a
// fixed LDS tree and writes one partial per (quantity, column); a one-workgroup
// kernel launched next sums the partials in a fixed order and runs a small
// "finalize" step on thread 0 (CG scalars, convergence flags).  Issuing a
// device-scope fence per workgroup instead (a "last workgroup" ticket) makes
// every workgroup write back its XCD's L2 and costs far more than the launch.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace amg {

__device__ __forceinline__ int ceil_div_dev(int a, int b) { return (a + b - 1) / b; }
__device__ __forceinline__ long ceil_div_dev_l(long a, long b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// per-column CG state kept in device memory
struct ColScal {
    double rho, alpha, beta, bb, tol2, rr, pq, rz;
    double rho_next;  // fused finalize: r.z of the latest residual, committed to rho by the update
    int conv, iters, bad, pad;
};

// What the host needs to steer a CG, written by the finalize kernels into
// pinned host memory (read after an event, no copy kernels).
struct Mail {
    int all_conv;
    int bad;
    int iters;       // largest iteration count over the columns
    int indefinite;
    int nlive;       // refinement: columns still refining
    int stagnated;
    int pad[2];
};

struct CgScal {
    ColScal s[16];
    int all_conv;
    int nb;          // live columns; columns >= nb are padding and stay frozen
    int indefinite;  // outer CG: p.q <= 0 or r.z <= 0 met on a live column
    int pad;
    Mail *mail;      // host-mapped mailbox of this CG
    void *xptr;      // where the CG accumulates its solution (set at start)
};

__device__ __forceinline__ void publish(CgScal *sc, int NBc) {
    int all = 1, bad = 0, it = 0;
    for (int c = 0; c < NBc; ++c) {
        all &= sc->s[c].conv;
        bad |= sc->s[c].bad;
        it = max(it, sc->s[c].iters);
    }
    sc->all_conv = all;
    Mail *m = sc->mail;
    m->iters = it;
    m->bad = bad;
    m->indefinite = sc->indefinite;
    m->all_conv = all;
}

__device__ __forceinline__ int xcd_block(int b, int nblk) {
    // Workgroups are dispatched round-robin over the XCDs; give each XCD a
    // contiguous run of row blocks so neighbouring rows share an L2.
    const int per = nblk / kXcd;
    return (b % kXcd) * per + b / kXcd;
}

// Columns per lane: a lane serves CV consecutive columns of the batch, so its
// gathers and stores are CV contiguous values.
template <int NB> constexpr int spmv_cv() { return NB >= 4 ? 4 : NB; }

// Lanes per row: NB / CV column groups x G lanes per (row, group), G a power
// of two chosen per matrix from its mean row length; LPR = (NB / CV) G <= 64.
struct Geo {
    int lg;   // log2 G
    int llpr; // log2 LPR
    __host__ __device__ int lpr() const { return 1 << llpr; }
    __host__ __device__ int rpb() const { return kBlock >> llpr; }
};

inline int ilog2(int x) {
    int l = 0;
    while ((1 << (l + 1)) <= x) ++l;
    return l;
}

// entries a lane loads together
constexpr int kSpmvUnroll = 4;

// G = next power of two >= (mean entries per row) / U, at most 64 / (NB / CV)
template <int NB> inline Geo make_geo(long nnz, long rows) {
    constexpr int NG = NB / spmv_cv<NB>();
    const double m = rows > 0 ? (double)nnz / (double)rows : 1.0;
    int g = 1;
    while (g < 64 && g < m / kSpmvUnroll) g <<= 1;
    while (g * NG > 64) g >>= 1;
    if (g < 1) g = 1;
    Geo geo;
    geo.lg = ilog2(g);
    geo.llpr = ilog2(g * NG);
    return geo;
}

// the geometry with G = 2^lg lanes per (row, column group)
template <int NB> inline Geo geo_from_lg(int lg) {
    Geo geo;
    geo.lg = lg;
    geo.llpr = lg + ilog2(NB / spmv_cv<NB>());
    return geo;
}

// largest log2 G a product on NB columns can take (LPR <= 64)
template <int NB> constexpr int max_lg() { return NB >= 4 ? 6 - (NB == 4 ? 0 : NB == 8 ? 1 : 2) : 6; }

// the autotuner's choice for this matrix, batch width and value type, else the default rule
template <int NB, typename T> inline Geo geo_for(const DCsr &A) {
    const int t = A.tuned_lg[ilog2(NB)][std::is_same_v<T, float> ? 1 : 0];
    return t >= 0 ? geo_from_lg<NB>(t) : make_geo<NB>(A.nnz, A.n);
}

template <int NV, int NB> struct Reducer {
    double *partial;    // [NV*NB][gridDim.x]
};

constexpr int pow2floor(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

// Block reduction of acc over the threads that serve the same columns: thread
// t serves column group t % NG (NG = NB / CV groups of CV consecutive columns;
// slot v of acc is column (t % NG) CV + v).  Each wavefront folds its lanes of
// one group by shuffles (xor offsets NG, 2 NG, .., 32), the wavefronts' sums are
// added in order through LDS, and thread t < NV NB writes partial (t / NB,
// t % NB) of this workgroup.  The totals are formed by fin_kernel, launched next
// on the same stream (a kernel boundary orders the partials; no device-scope
// fence is issued by the workgroups).
template <int NV, int NB, int CV>
__device__ void block_partials_cv(const double (&acc)[CV][NV], Reducer<NV, NB> r) {
    constexpr int NG = NB / CV, WV = kBlock / 64;
    __shared__ double wred[WV][NV][NB];
    const int t = threadIdx.x, lane = t & 63;
#pragma unroll
    for (int v = 0; v < CV; ++v)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double x = acc[v][q];
#pragma unroll
            for (int off = NG; off < 64; off <<= 1) x += __shfl_xor(x, off);
            if (lane < NG) wred[t >> 6][q][lane * CV + v] = x;
        }
    __syncthreads();
    if (t < NV * NB) {
        double x = 0.0;
#pragma unroll
        for (int w = 0; w < WV; ++w) x += wred[w][t / NB][t % NB];
        r.partial[(size_t)t * gridDim.x + blockIdx.x] = x;
    }
}

template <int NV, int NB>
__device__ void block_partials(const double (&acc)[NV], Reducer<NV, NB> r) {
    const double(&a1)[1][NV] = *reinterpret_cast<const double(*)[1][NV]>(&acc);
    block_partials_cv<NV, NB, 1>(a1, r);
}

// Sums the partials of Q quantities in a fixed order with all BS threads of
// the workgroup: quantity q's partials are src(q, &ptr, &count).  LPS threads
// (a power of two) serve a quantity: each keeps eight running sums over the
// partials it strides through (eight loads in flight), then the LPS sums are
// folded by wavefront shuffles and, for LPS > 64, across the quantity's
// wavefronts through LDS.  The order depends only on the counts, so every
// workgroup that sums the same partials gets the same totals.  out (LDS,
// [Q]) holds the totals for every thread on return.
template <int Q, int BS, class SRC>
__device__ void sum_quantities(SRC src, double *out) {
    constexpr int LPS = pow2floor(BS / Q);
    constexpr int W = LPS < 64 ? LPS : 64;
    __shared__ double wsum[BS / 64];
    const int t = threadIdx.x;
    const int q = t / LPS, sub = t % LPS;
    double s = 0.0;
    if (q < Q) {
        const double *pp;
        int nblk;
        src(q, pp, nblk);
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int b = sub;
        for (; b + 7 * LPS < nblk; b += 8 * LPS) {
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = pp[b + k * LPS];
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] += v[k];
        }
        // at most seven left: loaded unconditionally (clamped index), added
        // only where valid, so the seven loads are in flight together
        const int last = nblk > 0 ? nblk - 1 : 0;
        double v[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] = pp[min(b + k * LPS, last)];
#pragma unroll
        for (int k = 0; k < 7; ++k) a[k] = b + k * LPS < nblk ? a[k] + v[k] : a[k];
        s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
#pragma unroll
    for (int off = W / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if constexpr (LPS > 64) {
        if ((t & 63) == 0) wsum[t >> 6] = s;
        __syncthreads();
        if (sub == 0 && q < Q) {
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < LPS / 64; ++w) v += wsum[(t >> 6) + w];
            out[q] = v;
        }
    } else {
        if (sub == 0 && q < Q) out[q] = s;
    }
    __syncthreads();
}

// The partials of NV quantities x NB columns, quantity-major ([NV*NB][nblk]).
template <int NV, int NB, int BS = kBlock>
__device__ void sum_partials(const double *__restrict__ partial, int nblk, double (&tot)[NV][NB]) {
    sum_quantities<NV * NB, BS>(
        [&](int q, const double *&pp, int &n) {
            pp = partial + (size_t)q * nblk;
            n = nblk;
        },
        &tot[0][0]);
}

// Two buffers of one quantity x NB columns each, summed together.
template <int NB, int BS = kBlock>
__device__ void sum_partials2(const double *__restrict__ pa, int na, const double *__restrict__ pb, int nb,
                              double (&ta)[1][NB], double (&tb)[1][NB]) {
    __shared__ double both[2 * NB];
    sum_quantities<2 * NB, BS>(
        [&](int q, const double *&pp, int &n) {
            if (q < NB) {
                pp = pa + (size_t)q * na;
                n = na;
            } else {
                pp = pb + (size_t)(q - NB) * nb;
                n = nb;
            }
        },
        both);
    if (threadIdx.x < NB) {
        ta[0][threadIdx.x] = both[threadIdx.x];
        tb[0][threadIdx.x] = both[NB + threadIdx.x];
    }
    __syncthreads();
}

// Convergence test and beta of one CG column after an update (r.r = rr) and
// the preconditioner (r.z = rz): the step of the finalize kernels, shared by
// the fused form below.  Returns the new beta (0 when the column stops).
__device__ __forceinline__ double cg_col_step(const ColScal &s, double rr, double rz, int &conv, int &bad) {
    conv = s.conv;
    bad = s.bad;
    if (conv) return 0.0;
    if (bad || rr <= s.tol2) {
        conv = 1;
        return 0.0;
    }
    if (!(rz > 0.0)) {
        bad = 1;
        conv = 1;
        return 0.0;
    }
    return rz / s.rho;
}

// The finalize of a captured CG iteration folded into the first kernel of the
// next one: every workgroup sums the partials of r.r (buffer p1, quantity 0)
// and r.z (Jacobi: p1, quantity 1; else buffer p2) in the same fixed order,
// so all reach the same beta and convergence decisions; workgroup 0 records
// them (rho_next = r.z, committed to rho by the update kernel that follows,
// so no workgroup here reads a value another one writes, conv and bad only
// ever switch on), counts the iteration and publishes the mailbox.
struct NoPro {
    static constexpr bool active = false;
};

template <int NB, bool JAC> struct FusedFin {
    static constexpr bool active = true;
    CgScal *sc;
    const double *p1;
    int n1;
    const double *p2;
    int n2;
};

// Returns whether every column has stopped; beta[c] (in LDS) holds the new betas.
template <int NB, bool JAC>
__device__ bool fused_fin(const FusedFin<NB, JAC> &f, const double *&beta) {
    __shared__ double t1[JAC ? 2 : 1][NB], t2[1][NB];
    __shared__ double sb[NB];
    __shared__ int sall;
    // the column scalars the step reads, loaded before the partial sums so that
    // both loads are in flight together (nothing written in this kernel
    // changes what the step decides from them: see above)
    ColScal pre[NB];  // conv, bad, tol2 and rho only
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            pre[c].conv = f.sc->s[c].conv;
            pre[c].bad = f.sc->s[c].bad;
            pre[c].tol2 = f.sc->s[c].tol2;
            pre[c].rho = f.sc->s[c].rho;
        }
    if constexpr (JAC) sum_partials<2, NB>(f.p1, f.n1, t1);
    else sum_partials2<NB>(f.p1, f.n1, f.p2, f.n2, t1, t2);
    if (threadIdx.x == 0) {
        int all = 1;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            ColScal &s = f.sc->s[c];
            const double rr = t1[0][c], rz = JAC ? t1[1][c] : t2[0][c];
            const int was = pre[c].conv;
            int conv, bad;
            const double b = cg_col_step(pre[c], rr, rz, conv, bad);
            if (blockIdx.x == 0 && !was) {
                s.iters += 1;
                s.rr = rr;
                s.rz = rz;
                s.beta = b;
                s.rho_next = rz;
                s.bad = bad;
                s.conv = conv;
            }
            sb[c] = b;
            all &= conv;
        }
        sall = all;
        if (blockIdx.x == 0) publish(f.sc, NB);
    }
    __syncthreads();
    beta = sb;
    return sall != 0;
}

// The same step as a finalize kernel (after the last update a CG is allowed).
template <int NB, bool JAC> struct FinFusedTail {
    CgScal *sc;
    __device__ void step(const double (&rr)[NB], const double (&rz)[NB]) const {
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            if (s.conv) continue;
            int conv, bad;
            const double b = cg_col_step(s, rr[c], rz[c], conv, bad);
            s.iters += 1;
            s.rr = rr[c];
            s.rz = rz[c];
            s.beta = b;
            s.rho_next = rz[c];
            s.bad = bad;
            s.conv = conv;
        }
        publish(sc, NB);
    }
    __device__ void operator()(double (&tot)[2][NB]) const { step(tot[0], tot[1]); }  // Jacobi
    __device__ void operator()(double (&rr)[1][NB], double (&rz)[1][NB]) const { step(rr[0], rz[0]); }
};

// Finalize functors that keep their CG's scalars in a member sc (CgScal *)
// run on a copy of them in LDS: the workgroup loads the block at once and
// writes it back after the step, so thread 0's loop over the columns makes
// no chain of dependent global loads (one per column and field before).
template <class F, class = void> struct fin_has_sc : std::false_type {};
template <class F>
struct fin_has_sc<F, std::void_t<decltype(std::declval<F &>().sc)>>
    : std::is_same<decltype(std::declval<F &>().sc), CgScal *> {};

constexpr int kScWords = (int)(sizeof(CgScal) / sizeof(unsigned long long));
static_assert(sizeof(CgScal) % sizeof(unsigned long long) == 0, "CgScal is copied in 8-byte words");

__device__ __forceinline__ unsigned long long sc_stage_load(const CgScal *sc) {
    const int t = threadIdx.x;
    return t < kScWords ? reinterpret_cast<const unsigned long long *>(sc)[t] : 0ull;
}

// the step on the LDS copy (loaded by sc_stage_load before the partial sums,
// so both loads are in flight together), then the copy back
template <class FIN, class STEP>
__device__ __forceinline__ void fin_staged(const FIN &fin, unsigned long long w, STEP step) {
    __shared__ CgScal lsc;
    const int t = threadIdx.x;
    if (t < kScWords) reinterpret_cast<unsigned long long *>(&lsc)[t] = w;
    __syncthreads();
    if (t == 0) {
        FIN f = fin;
        f.sc = &lsc;
        step(f);
    }
    __syncthreads();
    if (t < kScWords) reinterpret_cast<unsigned long long *>(fin.sc)[t] = reinterpret_cast<unsigned long long *>(&lsc)[t];
}

// One workgroup: totals of the partials, then the finalize step on thread 0.
template <int NV, int NB, class FIN>
__global__ __launch_bounds__(kFinBlock) void fin_kernel(const double *__restrict__ partial, int nblk, FIN fin,
                                                        const int *__restrict__ stop) {
    if (stop && *stop) return;
    __shared__ double tot[NV][NB];
    if constexpr (fin_has_sc<FIN>::value) {
        const unsigned long long w = sc_stage_load(fin.sc);
        sum_partials<NV, NB, kFinBlock>(partial, nblk, tot);
        fin_staged(fin, w, [&](const FIN &f) { f(tot); });
    } else {
        sum_partials<NV, NB, kFinBlock>(partial, nblk, tot);
        if (threadIdx.x == 0) fin(tot);
    }
}

// The same with two partial buffers (one quantity each).
template <int NB, class FIN>
__global__ __launch_bounds__(kFinBlock) void fin2_kernel(const double *__restrict__ pa, int na,
                                                         const double *__restrict__ pb, int nb, FIN fin,
                                                         const int *__restrict__ stop) {
    if (stop && *stop) return;
    __shared__ double ta[1][NB], tb[1][NB];
    if constexpr (fin_has_sc<FIN>::value) {
        const unsigned long long w = sc_stage_load(fin.sc);
        sum_partials2<NB, kFinBlock>(pa, na, pb, nb, ta, tb);
        fin_staged(fin, w, [&](const FIN &f) { f(ta, tb); });
    } else {
        sum_partials2<NB, kFinBlock>(pa, na, pb, nb, ta, tb);
        if (threadIdx.x == 0) fin(ta, tb);
    }
}

struct NoFin {
    template <int NV, int NB> __device__ void operator()(double (&)[NV][NB]) const {}
};

// ---------------------------------------------------------------------------
// CSR SpMV / SpMM with a gather functor (how x_k is formed) and an epilogue
// functor (what is written for row i); optional fused reductions.
// FINE = 1 marks launches on the finest level (a separate instantiation, so that
// profiles separate the fine-level kernels from the coarse-level ones).
template <typename T, int NB, int NV, class GX, class EP, int FINE, class PRO = NoPro>
__global__ __launch_bounds__(kBlock) void spmv_kernel(int nrows, const int *__restrict__ rp,
                                                      const int *__restrict__ ci,
                                                      const T *__restrict__ av, GX gx, EP ep, Geo geo,
                                                      Reducer<(NV > 0 ? NV : 1), NB> red,
                                                      const int *__restrict__ stop, PRO pro = PRO{}) {
    if (stop && *stop) return;
    constexpr int CV = spmv_cv<NB>(), NG = NB / CV;
    const int t = threadIdx.x;
    const int LPR = geo.lpr(), RPB = geo.rpb(), G = 1 << geo.lg;
    const int lane = t & (LPR - 1), c0 = (lane % NG) * CV, g = lane / NG, rl = t >> geo.llpr;
    const int nblk = gridDim.x, b = xcd_block(blockIdx.x, nblk);
    const int span = ceil_div_dev(nrows, nblk * RPB) * RPB;
    const int r0 = b * span;
    const int r1 = min(nrows, r0 + span);
    GX gxv[CV];
    EP epv[CV];
#pragma unroll
    for (int v = 0; v < CV; ++v) {
        gxv[v] = gx;
        gxv[v].prep(c0 + v);
        epv[v] = ep;
        epv[v].prep(c0 + v);
    }
    if constexpr (PRO::active) {  // the previous iteration's finalize, then this one
        const double *fb;
        if (fused_fin(pro, fb)) return;
#pragma unroll
        for (int v = 0; v < CV; ++v) {
            gxv[v].set_beta(fb[c0 + v]);
            epv[v].set_beta(fb[c0 + v]);
        }
    }
    constexpr int NVA = NV > 0 ? NV : 1;
    double acc[CV][NVA];
#pragma unroll
    for (int v = 0; v < CV; ++v)
#pragma unroll
        for (int q = 0; q < NVA; ++q) acc[v][q] = 0.0;
    constexpr int U = kSpmvUnroll;  // entries per lane issued together
    for (int base = r0; base < r1; base += RPB) {
        const int row = base + rl;
        const bool live = row < r1;
        typename EP::P pr[CV];
        if (live && g == 0) {
#pragma unroll
            for (int v = 0; v < CV; ++v) pr[v] = epv[v].load(row, c0 + v);
        }
        T sum[CV];
#pragma unroll
        for (int v = 0; v < CV; ++v) sum[v] = T(0);
        if (live) {
            const int p1 = rp[row + 1];
            for (int p = rp[row] + g; p < p1; p += U * G) {
                // unconditional loads (past the row's end: its last entry,
                // weighted by 0), so all U loads and gathers are in flight together
                int kk[U];
                T aa[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = p + u * G;
                    const int qc = min(q, p1 - 1);
                    kk[u] = ci[qc];
                    const T a = av[qc];
                    aa[u] = q < p1 ? a : T(0);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int v = 0; v < CV; ++v) sum[v] += aa[u] * gxv[v](kk[u], c0 + v);
                }
            }
        }
        for (int off = NG; off < LPR; off <<= 1) {
#pragma unroll
            for (int v = 0; v < CV; ++v) sum[v] += __shfl_xor(sum[v], off);
        }
        if (live && g == 0) {
#pragma unroll
            for (int v = 0; v < CV; ++v) epv[v](row, c0 + v, sum[v], pr[v], acc[v]);
        }
    }
    if constexpr (NV > 0) block_partials_cv<NV, NB, CV>(acc, red);
}

// The same product over the sliced-ELL copy (single column): one wavefront
// per slice of 64 rows, one lane per row; a lane issues the loads of up to U
// entries of its row at once, with no dependence on row pointers (U = 8 when
// no slice is wider, as for 5- and 7-point rows, else 16).  Columns are
// 16-bit offsets from the slice's base column (6 bytes per float32 entry).
// xrot rotates the XCD-contiguous block ranges by xrot XCDs (0 in solves).
template <typename T, int NV, class GX, class EP, class PRO = NoPro, int U = 16>
__global__ __launch_bounds__(kBlock) void sell_kernel(int nrows, int nsl, const int *__restrict__ soff,
                                                      const int *__restrict__ sbase,
                                                      const uint16_t *__restrict__ cd, const T *__restrict__ av, GX gx,
                                                      EP ep, Reducer<(NV > 0 ? NV : 1), 1> red,
                                                      const int *__restrict__ stop, PRO pro = PRO{}, int xrot = 0) {
    if (stop && *stop) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nblk = gridDim.x, b = (xcd_block(blockIdx.x, nblk) + xrot * (nblk / kXcd)) % nblk;
    constexpr int WPB = kBlock / 64;
    const int per = ceil_div_dev(nsl, nblk * WPB) * WPB;  // contiguous slices per workgroup
    const int s0 = b * per, s1 = min(nsl, s0 + per);
    gx.prep(0);
    ep.prep(0);
    if constexpr (PRO::active) {  // the previous iteration's finalize, then this one
        const double *fb;
        if (fused_fin(pro, fb)) return;
        gx.set_beta(fb[0]);
        ep.set_beta(fb[0]);
    }
    constexpr int NVA = NV > 0 ? NV : 1;
    double acc[NVA];
#pragma unroll
    for (int v = 0; v < NVA; ++v) acc[v] = 0.0;
    for (int sl = s0 + wv; sl < s1; sl += WPB) {
        const int row = sl * 64 + lane;
        const bool live = row < nrows;
        typename EP::P pr{};
        if (live) pr = ep.load(row, 0);
        const int o = soff[sl], w = (soff[sl + 1] - o) >> 6, cb = sbase[sl];
        T sum = T(0);
        for (int k0 = 0; k0 < w; k0 += U) {
            // Every load is unconditional (entries past the slice's width read
            // its last entry again, weighted by 0), so the U column and value
            // loads, then the U gathers, are in flight together; guarded loads
            // compile to one wait per entry.  A weight of exactly 0 leaves the
            // sum unchanged.
            int kk[U];
            T aa[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t q = (size_t)o + (size_t)min(k0 + u, w - 1) * 64 + lane;
                kk[u] = cb + (int)cd[q];
                const T a = av[q];
                aa[u] = k0 + u < w ? a : T(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) sum += aa[u] * gx(kk[u], 0);
        }
        if (live) ep(row, 0, sum, pr, acc);
    }
    if constexpr (NV > 0) block_partials<NV, 1>(acc, red);
}

// Elementwise kernel over n rows x NB columns with fused reductions.
template <int NB, int NV, class OP, int FINE>
__global__ __launch_bounds__(kBlock) void elem_kernel(int n, OP op, Reducer<(NV > 0 ? NV : 1), NB> red,
                                                      const int *__restrict__ stop) {
    if (stop && *stop) return;
    const int t = threadIdx.x, c = t % NB;
    const int nblk = gridDim.x, b = xcd_block(blockIdx.x, nblk);
    const long total = (long)n * NB;
    const long span = (long)ceil_div_dev_l(total, (long)nblk * kBlock) * kBlock;
    const long e0 = (long)b * span;
    const long e1 = total < e0 + span ? total : e0 + span;
    op.prep(c);
    constexpr int NVA = NV > 0 ? NV : 1;
    double acc[NVA];
#pragma unroll
    for (int v = 0; v < NVA; ++v) acc[v] = 0.0;
    for (long e = e0 + t; e < e1; e += kBlock) op((int)(e / NB), c, acc);
    if constexpr (NV > 0) block_partials<NV, NB>(acc, red);
}

// CG update: every workgroup first sums the p.q partials of the preceding
// operator kernel (same fixed order in all workgroups, so all agree on alpha),
// then x += alpha p, r -= alpha q (Jacobi: z = dinv r) on the live columns,
// with the partials of r.r (and r.z).  Workgroup 0 records alpha and flags a
// non-positive p.q (breakdown, or indefiniteness for the outer CG).
template <typename T, int NB, bool JAC, int FINE>
__global__ __launch_bounds__(kBlock) void cg_update_kernel(int n, T *__restrict__ x, T *__restrict__ r,
                                                           T *__restrict__ z, float *__restrict__ r32,
                                                           float *__restrict__ x32, const float *__restrict__ d32,
                                                           double s0, int fused,
                                                           const T *__restrict__ p,
                                                           const T *__restrict__ q, const T *__restrict__ dinv,
                                                           CgScal *sc, const double *__restrict__ part_pq,
                                                           int nblk_pq, int outer,
                                                           Reducer<JAC ? 2 : 1, NB> red,
                                                           const int *__restrict__ stop) {
    if (stop && *stop) return;
    if (!x) x = static_cast<T *>(sc->xptr);
    __shared__ double pq[1][NB];
    __shared__ double sh_a[NB];
    __shared__ int sh_live[NB];
    const int t = threadIdx.x;
    // the column's scalars, loaded before the partial sums so that both loads
    // are in flight together (workgroup 0 writes only fields read here by no one)
    int conv0 = 0;
    double rho0 = 0.0;
    if (t < NB) {
        conv0 = sc->s[t].conv;
        rho0 = fused ? sc->s[t].rho_next : sc->s[t].rho;
    }
    if (nblk_pq > 0) sum_partials<1, NB>(part_pq, nblk_pq, pq);
    if (nblk_pq == 0) {
        // alpha was formed by a finalize kernel (many partials)
        if (t < NB) {
            sh_a[t] = sc->s[t].alpha;
            sh_live[t] = !conv0;
        }
    } else if (t < NB) {
        ColScal &s = sc->s[t];
        const double v = pq[0][t];
        double a = 0.0;
        int live = !conv0;
        if (live) {
            if (v > 0.0) {
                a = rho0 / v;
            } else {
                live = 0;
                if (blockIdx.x == 0) {
                    s.bad = 1;
                    if (outer) sc->indefinite = 1;
                }
            }
        }
        sh_a[t] = a;
        sh_live[t] = live;
        if (blockIdx.x == 0) {
            s.alpha = a;
            s.pq = v;
            if (fused && !conv0) s.rho = rho0;
        }
    }
    __syncthreads();
    const int c = t % NB;
    const T a = (T)sh_a[c];
    const int live = sh_live[c];
    const int nblk = gridDim.x, b = xcd_block(blockIdx.x, nblk);
    const long total = (long)n * NB;
    const long span = (long)ceil_div_dev_l(total, (long)nblk * kBlock) * kBlock;
    const long e0 = (long)b * span;
    const long e1 = total < e0 + span ? total : e0 + span;
    double acc[JAC ? 2 : 1] = {};
    if (live) {
        for (long e = e0 + t; e < e1; e += kBlock) {
            const size_t o = (size_t)e;
            x[o] += a * p[o];
            const T rv = r[o] - a * q[o];
            r[o] = rv;
            acc[0] += (double)rv * (double)rv;
            if constexpr (JAC) {
                const T zz = dinv[e / NB] * rv;
                z[o] = zz;
                acc[1] += (double)rv * (double)zz;
            } else {
                // the V-cycle's first pre-sweep iterate x0 = D^{-1} r (in its precision)
                if (z) z[o] = (dinv[e / NB] * rv) * (T)s0;
                if (r32) {
                    const float rf = (float)rv;
                    r32[o] = rf;
                    if (x32) x32[o] = (d32[e / NB] * rf) * (float)s0;
                }
            }
        }
    }
    block_partials<JAC ? 2 : 1, NB>(acc, red);
}

// ---------------------------------------------------------------------------
// gathers
template <typename T, int NB> struct GPlain {  // x_k
    const T *x;
    __device__ void prep(int) {}
    __device__ T operator()(int k, int c) const { return x[(size_t)k * NB + c]; }
};

template <typename T, int NB, typename TZ = T> struct GZBP {  // p_k = z_k + beta_c pold_k
    const TZ *z;
    const T *pold;
    const CgScal *sc;
    T beta;
    __device__ void prep(int c) { beta = (T)sc->s[c].beta; }
    __device__ void set_beta(double b) { beta = (T)b; }
    __device__ T operator()(int k, int c) const {
        return (T)z[(size_t)k * NB + c] + beta * pold[(size_t)k * NB + c];
    }
};

// z_k alone: the CG product formed as A z + beta q_old (ECgQR)
template <typename T, int NB, typename TZ = T> struct GZ {
    const TZ *z;
    __device__ void prep(int) {}
    __device__ void set_beta(double) {}
    __device__ T operator()(int k, int c) const { return (T)z[(size_t)k * NB + c]; }
};

// x_k = keep_k a_k + s b_k with keep_k = (mask == null || mask[k] == 0)
template <int NB> struct GLin {
    const double *a;
    const uint8_t *mask;
    const double *b;
    double s;
    __device__ void prep(int) {}
    __device__ double operator()(int k, int c) const {
        double v = a[(size_t)k * NB + c];
        if (mask && mask[k]) v = 0.0;
        if (b) v += s * b[(size_t)k * NB + c];
        return v;
    }
};

// ---------------------------------------------------------------------------
// epilogues: load(i, c) fetches the row's own operands before the entry loop
// (so their latency overlaps the gathers); operator() then writes the row.
struct NoPre {};

template <typename T, int NB> struct EStore {  // y_i = sum
    T *y;
    using P = NoPre;
    __device__ void prep(int) {}
    __device__ P load(int, int) const { return {}; }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &, double (&)[NV]) const {
        y[(size_t)i * NB + c] = s;
    }
};

template <typename T, int NB> struct EAdd {  // y_i += sum
    T *y;
    struct P {
        T y0;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const { return {y[(size_t)i * NB + c]}; }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &pr, double (&)[NV]) const {
        y[(size_t)i * NB + c] = pr.y0 + s;
    }
};

// residual after the first pre-sweep, whose iterate x = dinv b the producer
// of b has written: r_i = b_i - (A x)_i
template <typename T, int NB> struct EResB {
    const T *b;
    T *r;
    struct P {
        T b;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const { return {b[(size_t)i * NB + c]}; }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &pr, double (&)[NV]) const {
        r[(size_t)i * NB + c] = pr.b - s;
    }
};

// restriction that also starts the next level's pre-smoothing: y_i = sum,
// x_i = (dinv_i sum) s0 (s0 = 1 for l1-Jacobi, 1/theta for Chebyshev)
template <typename T, int NB> struct EStoreX {
    T *y;
    const T *dinv;
    T *x;
    T s0;
    struct P {
        T d;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int) const { return {dinv[i]}; }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &pr, double (&)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        y[o] = s;
        x[o] = (pr.d * s) * s0;
    }
};

// Chebyshev smoothing (degree 2, l1 diagonal), second step from the first
// iterate x1 = (dinv b) / theta: out_i = x1_i + (c1 x1_i + c2 dinv_i (b_i - (A x1)_i))
template <typename T, int NB> struct EChebPre {
    const T *b;
    const T *dinv;
    const T *x1;
    T *out;
    T c1, c2;
    struct P {
        T b, d, x;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const {
        const size_t o = (size_t)i * NB + c;
        return {b[o], dinv[i], x1[o]};
    }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &pr, double (&)[NV]) const {
        const T r = pr.d * (pr.b - s);
        const T d = c1 * pr.x + c2 * r;
        out[(size_t)i * NB + c] = pr.x + d;
    }
};

// Chebyshev smoothing from an iterate y0, first step:
// y1_i = y0_i + (dinv_i (b_i - (A y0)_i)) s0
template <typename T, int NB> struct EChebPost1 {
    const T *b;
    const T *dinv;
    const T *y0;
    T *y1;
    T s0;
    struct P {
        T b, d, y;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const {
        const size_t o = (size_t)i * NB + c;
        return {b[o], dinv[i], y0[o]};
    }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &pr, double (&)[NV]) const {
        y1[(size_t)i * NB + c] = pr.y + (pr.d * (pr.b - s)) * s0;
    }
};

// second step: out_i = y1_i + (c1 (y1_i - y0_i) + c2 dinv_i (b_i - (A y1)_i));
// optionally acc += b_i out_i
template <typename T, int NB, bool DOT> struct EChebPost2 {
    const T *b;
    const T *dinv;
    const T *y0;
    const T *y1;
    T *out;
    T c1, c2;
    struct P {
        T b, d, y0, y1;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const {
        const size_t o = (size_t)i * NB + c;
        return {b[o], dinv[i], y0[o], y1[o]};
    }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &pr, double (&acc)[NV]) const {
        const T r = pr.d * (pr.b - s);
        const T d = c1 * (pr.y1 - pr.y0) + c2 * r;
        const T v = pr.y1 + d;
        out[(size_t)i * NB + c] = v;
        if constexpr (DOT) acc[0] += (double)pr.b * (double)v;
    }
};

// post-smoothing: out_i = x_i + dinv_i (b_i - (A x)_i); optionally acc += b_i out_i
template <typename T, int NB, bool DOT> struct EPost {
    const T *dinv;
    const T *b;
    const T *x;
    T *out;
    struct P {
        T b, x, d;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const {
        const size_t o = (size_t)i * NB + c;
        return {b[o], x[o], dinv[i]};
    }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &pr, double (&acc)[NV]) const {
        const T v = pr.x + pr.d * (pr.b - s);
        out[(size_t)i * NB + c] = v;
        if constexpr (DOT) acc[0] += (double)pr.b * (double)v;
    }
};

// Prolongation fused into the first post-smoothing step.  The corrected
// iterate x + S e and the residual it leaves, b - A (x + S e) = r - T e with
// r = b - A x from the pre-smoothing and T = A S (the Galerkin intermediate,
// whose pattern contains that of S), come from one pass over T's pattern that
// carries S's values aligned to it (zero where S has no entry): per row i and
// column c, se = (S e)_i and te = (T e)_i, both gathered from the coarse
// vector e.  LPR = G NB lanes per row: G groups over the entries, one lane per
// column; the epilogue receives both sums.  Columns are int32 or, when the
// coarse level has at most 65536 nodes, 16-bit (CI = uint16_t).
template <typename T, int NB, int NV, class EP, typename CI = int>
__global__ __launch_bounds__(kBlock) void tpro_kernel(int nrows, const int *__restrict__ rp,
                                                      const CI *__restrict__ ci, const T *__restrict__ tv,
                                                      const T *__restrict__ sv, const T *__restrict__ e, EP ep,
                                                      int llpr, Reducer<(NV > 0 ? NV : 1), NB> red,
                                                      const int *__restrict__ stop) {
    if (stop && *stop) return;
    const int t = threadIdx.x, LPR = 1 << llpr, RPB = kBlock >> llpr, G = LPR / NB;
    const int lane = t & (LPR - 1), c = lane % NB, g = lane / NB, rl = t >> llpr;
    const int nblk = gridDim.x, b = xcd_block(blockIdx.x, nblk);
    const int span = ceil_div_dev(nrows, nblk * RPB) * RPB;
    const int r0 = b * span, r1 = min(nrows, r0 + span);
    EP epv = ep;
    epv.prep(c);
    constexpr int NVA = NV > 0 ? NV : 1;
    double acc[NVA];
#pragma unroll
    for (int q = 0; q < NVA; ++q) acc[q] = 0.0;
    constexpr int U = kSpmvUnroll;
    for (int base = r0; base < r1; base += RPB) {
        const int row = base + rl;
        const bool live = row < r1;
        typename EP::P pr{};
        if (live && g == 0) pr = epv.load(row, c);
        T se = T(0), te = T(0);
        if (live) {
            const int p1 = rp[row + 1];
            for (int p = rp[row] + g; p < p1; p += U * G) {
                // unconditional loads, as in spmv_kernel
                int kk[U];
                T ta[U], sa[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = p + u * G;
                    const int qc = min(q, p1 - 1);
                    kk[u] = (int)ci[qc];
                    const T a = tv[qc], s = sv[qc];
                    ta[u] = q < p1 ? a : T(0);
                    sa[u] = q < p1 ? s : T(0);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const T ev = e[(size_t)kk[u] * NB + c];
                    se += sa[u] * ev;
                    te += ta[u] * ev;
                }
            }
        }
        for (int off = NB; off < LPR; off <<= 1) {  // the G groups of a row and column
            se += __shfl_xor(se, off);
            te += __shfl_xor(te, off);
        }
        if (live && g == 0) epv(row, c, se, te, pr, acc);
    }
    if constexpr (NV > 0) block_partials<NV, NB>(acc, red);
}

// Chebyshev, first post step: y0 = t + S e (in place of t),
// y1 = y0 + (dinv (r - T e)) s0, i.e. y0 + (dinv (b - A y0)) s0
template <typename T, int NB> struct EProCheb {
    T *t;
    const T *r;
    const T *dinv;
    T *y1;
    T s0;
    struct P {
        T t, r, d;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const {
        const size_t o = (size_t)i * NB + c;
        return {t[o], r[o], dinv[i]};
    }
    template <int NV>
    __device__ void operator()(int i, int c, T se, T te, const P &pr, double (&)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        const T y0 = pr.t + se;
        t[o] = y0;
        y1[o] = y0 + (pr.d * (pr.r - te)) * s0;
    }
};

// l1-Jacobi post-sweep: out = (x + S e) + dinv (r - T e), i.e.
// x1 + dinv (b - A x1) with x1 = x + S e; optionally acc += b out
template <typename T, int NB, bool DOT> struct EProJac {
    const T *x;
    const T *r;
    const T *b;
    const T *dinv;
    T *out;
    struct P {
        T x, r, b, d;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const {
        const size_t o = (size_t)i * NB + c;
        return {x[o], r[o], DOT ? b[o] : T(0), dinv[i]};
    }
    template <int NV>
    __device__ void operator()(int i, int c, T se, T te, const P &pr, double (&acc)[NV]) const {
        const T x1 = pr.x + se;
        const T v = x1 + pr.d * (pr.r - te);
        out[(size_t)i * NB + c] = v;
        if constexpr (DOT) acc[0] += (double)pr.b * (double)v;
    }
};

// CG search direction and operator: p_i = z_i + beta pold_i, q_i = (A p)_i, acc p.q
template <typename T, int NB, typename TZ = T> struct ECgQ {
    const TZ *z;
    const T *pold;
    T *p;
    T *q;
    const CgScal *sc;
    T beta;
    struct P {
        T z, po;
    };
    __device__ void prep(int c) { beta = (T)sc->s[c].beta; }
    __device__ void set_beta(double b) { beta = (T)b; }
    __device__ P load(int i, int c) const {
        const size_t o = (size_t)i * NB + c;
        return {(T)z[o], pold[o]};
    }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &pr, double (&acc)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        const T pi = pr.z + beta * pr.po;
        p[o] = pi;
        q[o] = s;
        acc[0] += (double)pi * (double)s;
    }
};

// CG direction and its product without gathering the direction:
// p_i = z_i + beta pold_i and q_i = (A z)_i + beta qold_i, which is (A p)_i
// since qold = A pold; q is updated in place (row i reads and writes only its
// own entry), and beta = 0 takes (A z)_i alone; acc p.q
template <typename T, int NB, typename TZ = T> struct ECgQR {
    const TZ *z;
    const T *pold;
    T *p;
    T *q;
    const CgScal *sc;
    T beta;
    struct P {
        T z, po, qo;
    };
    __device__ void prep(int c) { beta = (T)sc->s[c].beta; }
    __device__ void set_beta(double b) { beta = (T)b; }
    __device__ P load(int i, int c) const {
        const size_t o = (size_t)i * NB + c;
        return {(T)z[o], pold[o], q[o]};
    }
    template <int NV> __device__ void operator()(int i, int c, T s, const P &pr, double (&acc)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        const T pi = pr.z + beta * pr.po;
        const T qi = beta != T(0) ? s + beta * pr.qo : s;
        p[o] = pi;
        q[o] = qi;
        acc[0] += (double)pi * (double)qi;
    }
};

// out_i = s1 keep_i sum + s2 y_i + s3 w_i (+ acc x_i out_i)
template <int NB> struct ELin {
    double *out;
    const uint8_t *mask;
    double s1;
    const double *y;
    double s2;
    const double *w;
    double s3;
    const double *dotx;  // acc[0] += dotx_i * out_i when not null
    struct P {
        double y0, w0, dx;
        int keep;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const {
        const size_t o = (size_t)i * NB + c;
        return {y ? y[o] : 0.0, w ? w[o] : 0.0, dotx ? dotx[o] : 0.0, !(mask && mask[i])};
    }
    template <int NV> __device__ void operator()(int i, int c, double s, const P &pr, double (&acc)[NV]) const {
        double v = pr.keep ? s1 * s : 0.0;
        if (y) v += s2 * pr.y0;
        if (w) v += s3 * pr.w0;
        out[(size_t)i * NB + c] = v;
        if (dotx) acc[0] += pr.dx * v;
    }
};

// residual for refinement: r_i = f_i - (A x)_i (FP64), acc r.r
template <int NB> struct EResid {
    const double *f;
    double *r;
    struct P {
        double f;
    };
    __device__ void prep(int) {}
    __device__ P load(int i, int c) const { return {f[(size_t)i * NB + c]}; }
    template <int NV> __device__ void operator()(int i, int c, double s, const P &pr, double (&acc)[NV]) const {
        const double v = pr.f - s;
        r[(size_t)i * NB + c] = v;
        acc[0] += v * v;
    }
};

// ---------------------------------------------------------------------------
// finalize steps (thread 0 of the last workgroup)
template <int NB> struct FinAlpha {  // alpha = rho / p.q on live columns
    CgScal *sc;
    int outer;  // 1: flag indefiniteness instead of treating it as breakdown
    int fused;  // 1: rho is the rho_next of the fused finalize, committed here
    __device__ void operator()(double (&tot)[1][NB]) const {
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            if (fused && !s.conv) s.rho = s.rho_next;
            s.pq = tot[0][c];
            if (s.conv) {
                s.alpha = 0.0;
                continue;
            }
            if (!(s.pq > 0.0)) {
                s.alpha = 0.0;
                s.bad = 1;
                if (outer) sc->indefinite = 1;
                s.conv = 1;
                continue;
            }
            s.alpha = s.rho / s.pq;
        }
        int all = 1;
        for (int c = 0; c < NB; ++c) all &= sc->s[c].conv;
        publish(sc, NB);
    }
};

template <int NB, bool JAC> struct FinUpd {  // convergence test on r.r (and Jacobi beta)
    CgScal *sc;
    __device__ void operator()(double (&tot)[JAC ? 2 : 1][NB]) const {
        int all = 1;
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            if (!s.conv) {
                s.iters += 1;
                s.rr = tot[0][c];
                if (s.rr <= s.tol2 || s.bad) s.conv = 1;
                if constexpr (JAC) {
                    const double rz = tot[1][c];
                    s.rz = rz;
                    s.beta = s.conv ? 0.0 : rz / s.rho;
                    s.rho = rz;
                }
            }
            all &= s.conv;
        }
        publish(sc, NB);
    }
};

// Inner V-cycle CG, once per iteration after the preconditioner: convergence
// test on r.r (partials of the update kernel), then beta from r.z (partials of
// the V-cycle's last kernel).
template <int NB> struct FinUB {
    CgScal *sc;
    __device__ void operator()(double (&rr)[1][NB], double (&rz)[1][NB]) const {
        int all = 1;
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            if (!s.conv) {
                s.iters += 1;
                s.rr = rr[0][c];
                if (s.bad || s.rr <= s.tol2) {
                    s.conv = 1;
                    s.beta = 0.0;
                } else {
                    const double v = rz[0][c];
                    if (!(v > 0.0)) {
                        s.bad = 1;
                        s.conv = 1;
                    } else {
                        s.rz = v;
                        s.beta = v / s.rho;
                        s.rho = v;
                    }
                }
            }
            all &= s.conv;
        }
        publish(sc, NB);
    }
};

// Inner V-cycle CG start: rho = r.z of the first preconditioner application.
template <int NB> struct FinRho0 {
    CgScal *sc;
    __device__ void operator()(double (&tot)[1][NB]) const {
        int all = 1;
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            s.beta = 0.0;
            if (!s.conv) {
                const double v = tot[0][c];
                if (!(v > 0.0)) {
                    s.bad = 1;
                    s.conv = 1;
                } else {
                    s.rho = v;
                    s.rz = v;
                }
            }
            all &= s.conv;
        }
        publish(sc, NB);
    }
};

template <int NB> struct FinBeta {  // beta = r.z / rho after the preconditioner
    CgScal *sc;
    int outer;
    __device__ void operator()(double (&tot)[1][NB]) const {
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            if (s.conv) {
                s.beta = 0.0;
                continue;
            }
            const double rz = tot[0][c];
            if (!(rz > 0.0)) {
                s.bad = 1;
                if (outer) sc->indefinite = 1;
                s.conv = 1;
                s.beta = 0.0;
                continue;
            }
            s.rz = rz;
            s.beta = rz / s.rho;
            s.rho = rz;
        }
        int all = 1;
        for (int c = 0; c < NB; ++c) all &= sc->s[c].conv;
        publish(sc, NB);
    }
};

// CG in the mass-matrix inner product (the coarsest Hessian level): after the
// preconditioner z = M^{-1} r, stop on r.z <= tol2 (tol2 = rtol^2 b.M^{-1}b, set
// by FinOuterInit from b.z), else beta = r.z / rho
template <int NB> struct FinRzConv {
    CgScal *sc;
    __device__ void operator()(double (&tot)[1][NB]) const {
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            if (s.conv) {
                s.beta = 0.0;
                continue;
            }
            const double rz = tot[0][c];
            s.iters += 1;
            s.rz = rz;
            s.rr = rz;
            if (s.bad || rz <= s.tol2) {
                s.conv = 1;
                s.beta = 0.0;
                continue;
            }
            if (!(rz > 0.0)) {
                s.bad = 1;
                s.conv = 1;
                s.beta = 0.0;
                continue;
            }
            s.beta = rz / s.rho;
            s.rho = rz;
        }
        publish(sc, NB);
    }
};

// initial state: bb = b.b, tol2 = rtol^2 bb, conv = (bb == 0); Jacobi: rho = r.z
template <int NB, bool JAC> struct FinInit {
    CgScal *sc;
    double rtol;
    int nlive;
    void *x;
    int fused;  // the first fused finalize then gives beta = 0, rho_next = r.z and iteration 0
    __device__ void operator()(double (&tot)[JAC ? 2 : 1][NB]) const {
        sc->xptr = x;
        sc->nb = nlive;
        int all = 1;
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            s.bb = tot[0][c];
            s.tol2 = rtol * rtol * s.bb;
            s.rr = s.bb;
            s.iters = 0;
            s.bad = 0;
            s.alpha = 0.0;
            s.beta = 0.0;
            s.rho = 1.0;
            s.conv = (c >= sc->nb) || !(s.bb > 0.0);
            if constexpr (JAC) {
                s.rz = tot[1][c];
                s.rho = s.conv ? 1.0 : s.rz;
            }
            if (fused) {
                s.rho = __builtin_huge_val();
                s.iters = -1;
            }
            all &= s.conv;
        }
        publish(sc, NB);
        sc->indefinite = 0;
    }
};

template <int NB> struct FinStore {  // plain reduction result into out[v*NB + c]
    double *out;
    template <int NV> __device__ void operator()(double (&tot)[NV][NB]) const {
        for (int v = 0; v < NV; ++v)
            for (int c = 0; c < NB; ++c) out[v * NB + c] = tot[v][c];
    }
};

// ---------------------------------------------------------------------------
// elementwise operations
// r = b, x = 0, pold = 0; Jacobi: z = dinv r; else, when z is given, the
// V-cycle's first pre-sweep iterate z = dinv r, and with r32 the float32
// residual and its iterate x32 = d32 r32
template <typename T, int NB, bool JAC> struct OpInit {
    const T *b;
    T *r, *x, *pold, *z;
    const T *dinv;
    float *r32;
    float *x32;
    const float *d32;
    double s0;  // scale of the first smoothing iterate (1, or 1/theta for Chebyshev)
    __device__ void prep(int) {}
    template <int NV> __device__ void operator()(int i, int c, double (&acc)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        const T v = b[o];
        r[o] = v;
        if constexpr (!JAC) {
            if (z) z[o] = (dinv[i] * v) * (T)s0;
            if (r32) {
                const float rf = (float)v;
                r32[o] = rf;
                if (x32) x32[o] = (d32[i] * rf) * (float)s0;
            }
        }
        x[o] = T(0);
        pold[o] = T(0);
        acc[0] += (double)v * (double)v;
        if constexpr (JAC) {
            const T zz = dinv[i] * v;
            z[o] = zz;
            acc[1] += (double)v * (double)zz;
        }
    }
};

template <typename T, int NB, bool JAC> struct OpUpd {  // x += a p, r -= a q (Jacobi: z = dinv r)
    T *x, *r, *z;
    const T *p, *q, *dinv;
    const CgScal *sc;
    T a;
    int live;
    __device__ void prep(int c) {
        a = (T)sc->s[c].alpha;
        live = !sc->s[c].conv;
    }
    template <int NV> __device__ void operator()(int i, int c, double (&acc)[NV]) const {
        if (!live) return;
        const size_t o = (size_t)i * NB + c;
        x[o] += a * p[o];
        const T rv = r[o] - a * q[o];
        r[o] = rv;
        acc[0] += (double)rv * (double)rv;
        if constexpr (JAC) {
            const T zz = dinv[i] * rv;
            z[o] = zz;
            acc[1] += (double)rv * (double)zz;
        }
    }
};

template <int NB> struct OpDot {  // acc[v] += x_v . y_v (up to 2 pairs)
    const double *x0, *y0, *x1, *y1;
    __device__ void prep(int) {}
    template <int NV> __device__ void operator()(int i, int c, double (&acc)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        acc[0] += x0[o] * y0[o];
        if constexpr (NV > 1) acc[1] += x1[o] * y1[o];
    }
};

template <int NB> struct OpAxpby {  // out = a x + b y (a, b per column or scalar), out may alias x or y
    double *out;
    const double *x, *y;
    double a, b;
    __device__ void prep(int) {}
    template <int NV> __device__ void operator()(int i, int c, double (&)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        double v = a * x[o];
        if (y) v += b * y[o];
        out[o] = v;
    }
};

// out = x - (y + b w)
template <int NB> struct OpSubSum {
    double *out;
    const double *x, *y, *w;
    double b;
    __device__ void prep(int) {}
    template <int NV> __device__ void operator()(int i, int c, double (&)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        out[o] = x[o] - (y[o] + b * w[o]);
    }
};

// outer CG direction update: p = z + beta_c p
template <int NB> struct OpPUpd {
    double *p;
    const double *z;
    const CgScal *sc;
    double beta;
    int live;
    __device__ void prep(int c) {
        beta = sc->s[c].beta;
        live = !sc->s[c].conv;
    }
    template <int NV> __device__ void operator()(int i, int c, double (&)[NV]) const {
        if (!live) return;
        const size_t o = (size_t)i * NB + c;
        p[o] = z[o] + beta * p[o];
    }
};

// FP64 refinement state per column, kept on the device
struct RefScal {
    double fn[16];  // ||f||
    double s[16];   // current ||r||
    int live[16];
    int nlive;
    int stagnated;
    double rtol;
    Mail *mail;     // host-mapped: nlive, stagnated
};

template <int NB> struct OpCopyNorm {  // r = f, x = 0, acc f.f
    const double *f;
    double *r, *x;
    __device__ void prep(int) {}
    template <int NV> __device__ void operator()(int i, int c, double (&acc)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        const double v = f[o];
        r[o] = v;
        x[o] = 0.0;
        acc[0] += v * v;
    }
};

template <int NB> struct FinRefInit {
    RefScal *rs;
    double rtol;
    int nlive;
    __device__ void operator()(double (&tot)[1][NB]) const {
        int nl = 0;
        rs->rtol = rtol;
        rs->stagnated = 0;
        for (int c = 0; c < 16; ++c) {
            const double fn = c < NB ? sqrt(tot[0][c]) : 0.0;
            rs->fn[c] = fn;
            rs->s[c] = fn;
            rs->live[c] = (c < nlive) && fn > 0.0;
            nl += rs->live[c];
        }
        rs->nlive = nl;
        rs->mail->nlive = nl;
        rs->mail->stagnated = rs->stagnated;
    }
};

// after r = f - A x: a live column finishes at ||r|| <= rtol ||f||; it has
// stagnated when the residual did not at least halve
template <int NB> struct FinRefine {
    RefScal *rs;
    __device__ void operator()(double (&tot)[1][NB]) const {
        int nl = 0;
        for (int c = 0; c < NB; ++c) {
            if (!rs->live[c]) continue;
            const double r = sqrt(tot[0][c]);
            if (r <= rs->rtol * rs->fn[c]) {
                rs->live[c] = 0;
                continue;
            }
            if (!(r <= 0.5 * rs->s[c])) rs->stagnated = 1;
            rs->s[c] = r;
            ++nl;
        }
        rs->nlive = nl;
        rs->mail->nlive = nl;
        rs->mail->stagnated = rs->stagnated;
    }
};

template <int NB> struct OpRefAdd {  // x64 += s_c d32 on live columns
    double *x;
    const float *d;
    const RefScal *rs;
    double sc;
    int on;
    __device__ void prep(int c) {
        sc = rs->s[c];
        on = rs->live[c];
    }
    template <int NV> __device__ void operator()(int i, int c, double (&)[NV]) const {
        if (!on) return;
        const size_t o = (size_t)i * NB + c;
        x[o] += sc * (double)d[o];
    }
};

template <int NB> struct OpCastScale {  // b32 = fp32(r / s_c), zero on finished columns
    float *b;
    const double *r;
    const RefScal *rs;
    double inv;
    __device__ void prep(int c) { inv = rs->live[c] ? 1.0 / rs->s[c] : 0.0; }
    template <int NV> __device__ void operator()(int i, int c, double (&)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        b[o] = (float)(r[o] * inv);
    }
};

// outer CG start: bb = b.b, rr = r.r
template <int NB> struct FinOuterInit {
    CgScal *sc;
    double rtol;
    int nlive;
    __device__ void operator()(double (&tot)[2][NB]) const {
        sc->nb = nlive;
        sc->indefinite = 0;
        int all = 1;
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            s.bb = tot[0][c];
            s.rr = tot[1][c];
            s.tol2 = rtol * rtol * s.bb;
            s.iters = 0;
            s.bad = 0;
            s.alpha = s.beta = 0.0;
            s.rho = 1.0;
            s.conv = (c >= nlive) || !(s.bb > 0.0) || s.rr <= s.tol2;
            all &= s.conv;
        }
        publish(sc, NB);
    }
};

template <int NB> struct FinRho {  // rho = r.z at the start of the outer CG
    CgScal *sc;
    __device__ void operator()(double (&tot)[1][NB]) const {
        for (int c = 0; c < NB; ++c) {
            ColScal &s = sc->s[c];
            if (s.conv) continue;
            const double rz = tot[0][c];
            if (!(rz > 0.0)) {
                s.bad = 1;
                sc->indefinite = 1;
                continue;
            }
            s.rho = rz;
            s.rz = rz;
        }
        publish(sc, NB);
    }
};

// V-cycle input from a packed FP64 vector: b = T(in) (zero on padding
// columns) and the first smoothing iterate x = (dinv b) s0 that the producer
// of a V-cycle's right-hand side writes
template <typename T, int NB> struct OpVcIn {
    T *b, *x;
    const double *in;
    const T *dinv;
    T s0;
    int nb;
    __device__ void prep(int) {}
    template <int NV> __device__ void operator()(int i, int c, double (&)[NV]) const {
        const size_t o = (size_t)i * NB + c;
        const T v = c < nb ? (T)in[(size_t)i * nb + c] : T(0);
        b[o] = v;
        if (x) x[o] = (dinv[i] * v) * s0;
    }
};

template <typename T, int NB> struct OpVcOut {  // out[i*nb + c] = double(z[i*NB + c]), c < nb
    double *out;
    const T *z;
    int nb;
    __device__ void prep(int) {}
    template <int NV> __device__ void operator()(int i, int c, double (&)[NV]) const {
        if (c < nb) out[(size_t)i * nb + c] = (double)z[(size_t)i * NB + c];
    }
};

template <int NB> struct OpPack {  // out[i*NB + c] = c < nb ? in[i*nb + c] : 0
    double *out;
    const double *in;
    int nb;
    __device__ void prep(int) {}
    template <int NV> __device__ void operator()(int i, int c, double (&)[NV]) const {
        out[(size_t)i * NB + c] = c < nb ? in[(size_t)i * nb + c] : 0.0;
    }
};

template <int NB> struct OpUnpack {  // out[i*nb + c] = in[i*NB + c], c < nb
    double *out;
    const double *in;
    int nb;
    __device__ void prep(int) {}
    template <int NV> __device__ void operator()(int i, int c, double (&)[NV]) const {
        if (c < nb) out[(size_t)i * nb + c] = in[(size_t)i * NB + c];
    }
};

// ---------------------------------------------------------------------------
// dense coarse-level apply: x = Inv b with Inv row-major (stride ld, a
// multiple of 64 entries, zero padded), entries TM (FP64 or float32), one
// wavefront per row, 16-byte loads four deep per lane, FP64 accumulation.
template <typename TM> struct Vec16;
template <> struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
    __device__ static double get(const double2 &v, int e) { return e == 0 ? v.x : v.y; }
};
template <> struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
    __device__ static double get(const float4 &v, int e) {
        return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
    }
};

// One column with b of the matrix's type and 16-byte aligned: b is read in the
// same 16-byte vectors as the matrix rows, eight vectors of each in flight per
// lane (a float32 row of up to 2048 entries is one round).  Every load is
// unconditional (guarded loads compile to a wait each): matrix vectors past the
// row's stride ld re-read its last vector and are zeroed, b vectors past its
// last full vector re-read that one and are zeroed, and the ragged last vector
// of b (b is not padded; the rows are zero-padded to ld) is read once per launch
// with clamped indices.  The products and their order are those of a guarded
// loop.
template <typename TM>
__global__ __launch_bounds__(kBlock) void dense_apply1_kernel(int n, int ld, const TM *__restrict__ inv,
                                                              const TM *__restrict__ b, TM *__restrict__ x,
                                                              const int *__restrict__ stop) {
    if (stop && *stop) return;
    using V = Vec16<TM>;
    using VT = typename V::type;
    constexpr int W = V::n, D = 8;
    const int lane = threadIdx.x % 64;
    const int w = (blockIdx.x * kBlock + threadIdx.x) / 64;
    const int nw = gridDim.x * kBlock / 64;
    const int nal = n - n % W;  // b's full vectors end here
    VT tail;                    // b[nal .. n-1], zeros after
    {
        TM t[W];
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const TM v = b[min(nal + e, n - 1)];
            t[e] = nal + e < n ? v : TM(0);
        }
        tail = *reinterpret_cast<const VT *>(t);
    }
    for (int i = w; i < n; i += nw) {
        double acc = 0.0;
        const TM *row = inv + (size_t)i * ld;
        for (int k0 = lane * W; k0 < n; k0 += 64 * W * D) {
            VT m[D], bv[D];
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const int k = k0 + u * 64 * W;
                const VT mv = *reinterpret_cast<const VT *>(row + min(k, ld - W));
                const VT bl = *reinterpret_cast<const VT *>(b + max(min(k, nal - W), 0));
                m[u] = k < n ? mv : VT{};
                bv[u] = k < nal ? bl : k == nal ? tail : VT{};
            }
            // keep the scheduler from interleaving the loads with their uses
            // (it would otherwise issue them one at a time)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < D; ++u)
#pragma unroll
                for (int e = 0; e < W; ++e) acc += V::get(m[u], e) * V::get(bv[u], e);
        }
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) x[i] = (TM)acc;
    }
}

template <typename T, typename TM, int NB>
__global__ __launch_bounds__(kBlock) void dense_apply_kernel(int n, int ld, const TM *__restrict__ inv,
                                                             const T *__restrict__ b, T *__restrict__ x,
                                                             const int *__restrict__ stop) {
    if (stop && *stop) return;
    using V = Vec16<TM>;
    using VT = typename V::type;
    constexpr int W = V::n, D = 4;
    const int lane = threadIdx.x % 64;
    const int w = (blockIdx.x * kBlock + threadIdx.x) / 64;
    const int nw = gridDim.x * kBlock / 64;
    for (int i = w; i < n; i += nw) {
        double acc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[c] = 0.0;
        const TM *row = inv + (size_t)i * ld;
        for (int k0 = lane * W; k0 < n; k0 += 64 * W * D) {
            // unconditional loads as in dense_apply1_kernel: entries past n
            // read a valid entry again and are weighted by 0
            VT m[D];
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const int k = k0 + u * 64 * W;
                const VT mv = *reinterpret_cast<const VT *>(row + min(k, ld - W));
                m[u] = k < n ? mv : VT{};
            }
#pragma unroll
            for (int u = 0; u < D; ++u) {
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const int k = k0 + u * 64 * W + e;
                    const double a = k < n ? V::get(m[u], e) : 0.0;
                    const size_t kc = (size_t)min(k, n - 1) * NB;
#pragma unroll
                    for (int c = 0; c < NB; ++c) acc[c] += a * (double)b[kc + c];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            double v = acc[c];
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
            acc[c] = v;
        }
        if (lane < NB) {
            double v = acc[0];
#pragma unroll
            for (int c = 1; c < NB; ++c)
                if (lane == c) v = acc[c];
            x[(size_t)i * NB + lane] = (T)v;
        }
    }
}

}  // namespace amg
