// Solve phase: V-cycle, inner CG (FP64, or float32 inside FP64 refinement),
// mass-matrix CG, Hessian action, the multilevel Hessian preconditioner in
// practical form and the outer CG (paper, Sections 2, 3.2 and 5.2).
//
// Every vector is [n x NB] with NB the padded batch width.  Columns converge
// and freeze independently.  Kernels of a CG iteration return at once when
// every column has converged, so the host only polls the convergence flags
// from the iteration count of the previous solve at that level onwards.
#pragma once

#include <algorithm>
#include <cmath>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "ctx.hpp"

namespace amg {

// Chebyshev smoothing of degree 2 with the l1 diagonal on the interval
// [kChebLo, kChebHi] of the spectrum of D_l1^{-1} A (its top is at most 1 on
// every level): first iterate from zero s0 dinv b, then steps
// d = c1 d + c2 dinv (b - A x), x += d (Chebyshev acceleration).
constexpr double kChebLo = 0.3, kChebHi = 1.0;
struct ChebConst {
    double s0, c1, c2;
};
inline ChebConst cheb_const() {
    const double theta = (kChebHi + kChebLo) / 2, delta = (kChebHi - kChebLo) / 2, sigma = theta / delta;
    const double rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
    return {1.0 / theta, rho1 * rho0, 2.0 * rho1 / delta};
}

// partials a fused finalize may sum in every workgroup of the next kernel
constexpr long kFusedPartials = 4096;

// A named range on the host timeline of a profiler (roctx), for the span of a scope.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

// Algorithmic bytes of one sparse product: row pointers, (column, value) per
// stored entry, the gathered vector once and the written one once, per column
// (int32 indices; the count of the method's work, whatever layout runs it).
inline double spmv_bytes(long n, long nnz, int val_bytes, int nb) {
    return 4.0 * (n + 1) + (4.0 + val_bytes) * (double)nnz + 2.0 * val_bytes * (double)n * nb;
}

template <int NB> struct Solver {
    Ctx &c;
    hipStream_t s;
    // reduction partials and polling events of this solver's stream (a solver
    // on the side stream has its own, so its CGs can run beside the main one)
    double **part;
    int *pgrid;
    hipEvent_t *pev;
    // XCD rotation of sliced-ELL launches (kernel timing only; 0 in solves)
    int xrot = 0;
    explicit Solver(Ctx &cc) : c(cc), s(cc.stream), part(cc.part), pgrid(cc.pgrid), pev(cc.poll_ev) {}
    Solver(Ctx &cc, hipStream_t st, double **pt, int *pg, hipEvent_t *ev)
        : c(cc), s(st), part(pt), pgrid(pg), pev(ev) {}

    // ---------------- launch helpers ----------------
    // Reductions write their partials into one of three buffers (pbuf) so that
    // a finalize kernel can combine the partials of two earlier kernels.
    template <int NV, class FIN> void finish(int pbuf, FIN fin, const int *stop) {
        if constexpr (NV > 0 && !std::is_same_v<FIN, NoFin>)
            hipLaunchKernelGGL((fin_kernel<NV, NB, FIN>), dim3(1), dim3(kFinBlock), 0, s, part[pbuf],
                               pgrid[pbuf], fin, stop);
    }

    // workgroups of a reducing product with A (the partials it leaves)
    template <typename T> int red_grid(const DCsr &A) const {
        if (NB == 1 && A.sl_off) return grid_rows(A.nsl, kBlock / 64, red_grid_max<NB>());
        return grid_rows(A.n, geo_for<NB, T>(A).rpb(), red_grid_max<NB>());
    }

    template <typename T, int NV, class GX, class EP, class FIN, class PRO = NoPro>
    void spmv(const DCsr &A, const T *vals, GX gx, EP ep, FIN fin, const int *stop, int pbuf = 0,
              PRO pro = PRO{}) {
        c.st.bytes += spmv_bytes(A.n, A.nnz, sizeof(T), NB);
        if constexpr (NB == 1) {
            const T *sv = nullptr;
            if constexpr (std::is_same_v<T, float>) sv = vals == A.v32 ? A.sl_v32 : nullptr;
            else sv = vals == A.v ? A.sl_v : nullptr;
            if (A.sl_off && sv) {
                const int g = grid_rows(A.nsl, kBlock / 64, NV > 0 ? red_grid_max<NB>() : kMaxGridPlain);
                Reducer<(NV > 0 ? NV : 1), NB> red{part[pbuf]};
                if (NV > 0) pgrid[pbuf] = g;
                if (!A.sl_over8)
                    hipLaunchKernelGGL((sell_kernel<T, NV, GX, EP, PRO, 8>), dim3(g), dim3(kBlock), 0, s, A.n,
                                       A.nsl, A.sl_off, A.sl_base, A.sl_cd, sv, gx, ep, red, stop, pro, xrot);
                else
                    hipLaunchKernelGGL((sell_kernel<T, NV, GX, EP, PRO, 16>), dim3(g), dim3(kBlock), 0, s, A.n,
                                       A.nsl, A.sl_off, A.sl_base, A.sl_cd, sv, gx, ep, red, stop, pro, xrot);
                finish<NV>(pbuf, fin, stop);
                return;
            }
        }
        const Geo geo = geo_for<NB, T>(A);
        const int g = grid_rows(A.n, geo.rpb(), NV > 0 ? red_grid_max<NB>() : kMaxGridPlain);
        Reducer<(NV > 0 ? NV : 1), NB> red{part[pbuf]};
        if (NV > 0) pgrid[pbuf] = g;
        if (A.n == c.N)
            hipLaunchKernelGGL((spmv_kernel<T, NB, NV, GX, EP, 1, PRO>), dim3(g), dim3(kBlock), 0, s, A.n, A.rp,
                               A.ci, vals, gx, ep, geo, red, stop, pro);
        else
            hipLaunchKernelGGL((spmv_kernel<T, NB, NV, GX, EP, 0, PRO>), dim3(g), dim3(kBlock), 0, s, A.n, A.rp,
                               A.ci, vals, gx, ep, geo, red, stop, pro);
        finish<NV>(pbuf, fin, stop);
    }

    // fused prolongation + first post-smoothing step at level Lv (tpro_kernel)
    template <typename T, int NV, class EP>
    void tpro(const Level &Lv, const T *e, EP ep, const int *stop, int pbuf = 0) {
        const DCsr &Tm = Lv.T;
        // the method's work here: the prolongation S e and the product A (x + S e)
        c.st.bytes += spmv_bytes(Lv.S.n, Lv.S.nnz, sizeof(T), NB) + spmv_bytes(Lv.A.n, Lv.A.nnz, sizeof(T), NB);
        const double m = Tm.n > 0 ? (double)Tm.nnz / (double)Tm.n : 1.0;
        int G = 1;
        const int tl = Tm.tuned_lg[ilog2(NB)][std::is_same_v<T, float> ? 1 : 0];
        if (tl >= 0) G = 1 << tl;  // the autotuner's choice
        else
            while (G * NB < 64 && G < m / kSpmvUnroll) G <<= 1;
        const int llpr = ilog2(G * NB);
        const int g = grid_rows(Tm.n, kBlock >> llpr, NV > 0 ? red_grid_max<NB>() : kMaxGridPlain);
        Reducer<(NV > 0 ? NV : 1), NB> red{part[pbuf]};
        if (NV > 0) pgrid[pbuf] = g;
        if (Lv.Tc16)
            hipLaunchKernelGGL((tpro_kernel<T, NB, NV, EP, uint16_t>), dim3(g), dim3(kBlock), 0, s, Tm.n, Tm.rp,
                               Lv.Tc16, avals<T>(Tm), tsvals<T>(Lv), e, ep, llpr, red, stop);
        else
            hipLaunchKernelGGL((tpro_kernel<T, NB, NV, EP>), dim3(g), dim3(kBlock), 0, s, Tm.n, Tm.rp, Tm.ci,
                               avals<T>(Tm), tsvals<T>(Lv), e, ep, llpr, red, stop);
    }

    template <int NV, class OP, class FIN> void elem(int n, OP op, FIN fin, const int *stop, int pbuf = 0) {
        const int g = grid_rows((long)n * NB, kBlock, NV > 0 ? red_grid_max<NB>() : kMaxGridPlain);
        Reducer<(NV > 0 ? NV : 1), NB> red{part[pbuf]};
        if (NV > 0) pgrid[pbuf] = g;
        if (n == c.N)
            hipLaunchKernelGGL((elem_kernel<NB, NV, OP, 1>), dim3(g), dim3(kBlock), 0, s, n, op, red, stop);
        else
            hipLaunchKernelGGL((elem_kernel<NB, NV, OP, 0>), dim3(g), dim3(kBlock), 0, s, n, op, red, stop);
        finish<NV>(pbuf, fin, stop);
    }

    // x += alpha p, r -= alpha q with alpha from the p.q partials in buffer 0;
    // r.r (and r.z) partials into buffer 1
    template <typename T, bool JAC>
    void cg_update(int n, T *x, T *r, T *z, const T *p, const T *q, const T *dinv, CgScal *sc, int outer,
                   const int *stop, float *r32 = nullptr, float *x32 = nullptr, const float *d32 = nullptr,
                   double s0 = 1.0, int fused = 0) {
        const int g = grid_rows((long)n * NB, kBlock, red_grid_max<NB>());
        Reducer<JAC ? 2 : 1, NB> red{part[1]};
        // alpha: every workgroup sums the p.q partials itself when they are few,
        // else one finalize kernel forms it first
        int nblk_pq = pgrid[0];
        if ((long)nblk_pq * NB > 2048) {
            finish<1>(0, FinAlpha<NB>{sc, outer, fused}, stop);
            nblk_pq = 0;
        }
        pgrid[1] = g;
        if (n == c.N)
            hipLaunchKernelGGL((cg_update_kernel<T, NB, JAC, 1>), dim3(g), dim3(kBlock), 0, s, n, x, r, z, r32, x32, d32, s0, fused, p, q, dinv,
                               sc, part[0], nblk_pq, outer, red, stop);
        else
            hipLaunchKernelGGL((cg_update_kernel<T, NB, JAC, 0>), dim3(g), dim3(kBlock), 0, s, n, x, r, z, r32, x32, d32, s0, fused, p, q, dinv,
                               sc, part[0], nblk_pq, outer, red, stop);
    }

    template <typename T> void dense_apply(const DenseOp &d, const T *b, T *x, const int *stop) {
        const int g = ceil_div((long)d.n * 64, kBlock);
        c.st.bytes += (double)sizeof(T) * ((double)d.n * d.n + 2.0 * d.n * NB);
        // the vector kernel reads b in 16-byte vectors: it needs one full vector
        if (NB == 1 && reinterpret_cast<uintptr_t>(b) % 16 == 0 && d.n * sizeof(T) >= 16) {
            const T *m;
            if constexpr (std::is_same_v<T, float>) m = d.m32;
            else m = d.m64;
            hipLaunchKernelGGL((dense_apply1_kernel<T>), dim3(g), dim3(kBlock), 0, s, d.n, d.ld, m, b, x, stop);
            return;
        }
        if constexpr (std::is_same_v<T, float>)
            hipLaunchKernelGGL((dense_apply_kernel<T, float, NB>), dim3(g), dim3(kBlock), 0, s, d.n, d.ld, d.m32, b,
                               x, stop);
        else
            hipLaunchKernelGGL((dense_apply_kernel<T, double, NB>), dim3(g), dim3(kBlock), 0, s, d.n, d.ld, d.m64,
                               b, x, stop);
    }

    void read_sc(const CgScal *d) {
        AMG_HIP(hipMemcpyAsync(c.hsc, d, sizeof(CgScal), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
    }

    void wait_mail() {
        AMG_HIP(hipEventRecord(pev[0], s));
        AMG_HIP(hipEventSynchronize(pev[0]));
    }

    template <typename T> CgWs<T> &inws(int l) {
        if constexpr (std::is_same_v<T, double>) return c.ws[l].in64;
        else return c.ws[l].in32;
    }

    // ---------------- V-cycle (AMG preconditioner for A_j) ----------------
    // z = V_j b: one l1-Jacobi sweep from zero, residual, restriction with
    // S^T, recursion, prolongation with S, one l1-Jacobi sweep; the cycle ends
    // with the dense inverse at the coarsest level or at the first coarser
    // level that holds one (n <= dense_solve_max).  With dot the last kernel
    // also writes the partials of r.z for the CG (b is the CG residual) to
    // buffer 2.  The first sweep's iterate x = D^{-1} b is written by whoever
    // produces b: the caller at level j (into the level's V-cycle x), the
    // restriction below it.
    // scale of the first smoothing iterate written by the producers of b
    double first_scale() const { return c.o.smoother == 1 ? cheb_const().s0 : 1.0; }

    template <typename T> void vcycle(int j, const T *b, T *z, bool dot, const int *stop) {
        const bool cheb = c.o.smoother == 1;
        const ChebConst cc = cheb_const();
        const T s0 = (T)first_scale(), c1 = (T)cc.c1, c2 = (T)cc.c2;
        int Lc = c.L - 1;
        for (int l = j + 1; l < c.L - 1; ++l)
            if (c.lev[l].Ainv) {
                Lc = l;
                break;
            }
        const T *bl = b;
        for (int l = j; l < Lc; ++l) {
            Level &Lv = c.lev[l];
            VcWs<T> &v = vcws<T>(c.ws[l]);
            if (cheb) {
                spmv<T, 0>(Lv.A, avals<T>(Lv.A), GPlain<T, NB>{v.x},
                           EChebPre<T, NB>{bl, dl1inv<T>(Lv), v.x, v.t, c1, c2}, NoFin{}, stop);
                spmv<T, 0>(Lv.A, avals<T>(Lv.A), GPlain<T, NB>{v.t}, EResB<T, NB>{bl, v.r}, NoFin{}, stop);
            } else {
                spmv<T, 0>(Lv.A, avals<T>(Lv.A), GPlain<T, NB>{v.x}, EResB<T, NB>{bl, v.r}, NoFin{}, stop);
            }
            VcWs<T> &vn = vcws<T>(c.ws[l + 1]);
            if (l + 1 < Lc)
                spmv<T, 0>(Lv.St, avals<T>(Lv.St), GPlain<T, NB>{v.r},
                           EStoreX<T, NB>{vn.b, dl1inv<T>(c.lev[l + 1]), vn.x, s0}, NoFin{}, stop);
            else
                spmv<T, 0>(Lv.St, avals<T>(Lv.St), GPlain<T, NB>{v.r}, EStore<T, NB>{vn.b}, NoFin{}, stop);
            T *bn = vn.b;
            bl = bn;
        }
        T *xc = (j == Lc) ? z : vcws<T>(c.ws[Lc]).x;
        dense_apply<T>(Lc == c.L - 1 ? c.dAc : c.lev[Lc].dA, bl, xc, stop);
        for (int l = Lc - 1; l >= j; --l) {
            Level &Lv = c.lev[l];
            VcWs<T> &v = vcws<T>(c.ws[l]);
            const T *e = (l + 1 == Lc) ? vcws<T>(c.ws[Lc]).x : vcws<T>(c.ws[l + 1]).x2;
            const T *bb = (l == j) ? b : v.b;
            T *out = (l == j) ? z : v.x2;
            // the coarse correction and the first post step in one pass over
            // T = A S (residual r - T e), when the level keeps T
            const bool fuse = Lv.T.rp && avals<T>(Lv.T) && tsvals<T>(Lv);
            if (cheb) {
                // the iterate is t; the first post step writes x, the second out
                if (fuse) {
                    tpro<T, 0>(Lv, e, EProCheb<T, NB>{v.t, v.r, dl1inv<T>(Lv), v.x, s0}, stop);
                } else {
                    spmv<T, 0>(Lv.S, avals<T>(Lv.S), GPlain<T, NB>{e}, EAdd<T, NB>{v.t}, NoFin{}, stop);
                    spmv<T, 0>(Lv.A, avals<T>(Lv.A), GPlain<T, NB>{v.t},
                               EChebPost1<T, NB>{bb, dl1inv<T>(Lv), v.t, v.x, s0}, NoFin{}, stop);
                }
                if (l == j && dot)
                    spmv<T, 1>(Lv.A, avals<T>(Lv.A), GPlain<T, NB>{v.x},
                               EChebPost2<T, NB, true>{bb, dl1inv<T>(Lv), v.t, v.x, out, c1, c2}, NoFin{}, stop, 2);
                else
                    spmv<T, 0>(Lv.A, avals<T>(Lv.A), GPlain<T, NB>{v.x},
                               EChebPost2<T, NB, false>{bb, dl1inv<T>(Lv), v.t, v.x, out, c1, c2}, NoFin{}, stop);
                continue;
            }
            if (fuse) {
                if (l == j && dot)
                    tpro<T, 1>(Lv, e, EProJac<T, NB, true>{v.x, v.r, bb, dl1inv<T>(Lv), out}, stop, 2);
                else
                    tpro<T, 0>(Lv, e, EProJac<T, NB, false>{v.x, v.r, bb, dl1inv<T>(Lv), out}, stop);
                continue;
            }
            spmv<T, 0>(Lv.S, avals<T>(Lv.S), GPlain<T, NB>{e}, EAdd<T, NB>{v.x}, NoFin{}, stop);
            if (l == j && dot)
                spmv<T, 1>(Lv.A, avals<T>(Lv.A), GPlain<T, NB>{v.x},
                           EPost<T, NB, true>{dl1inv<T>(Lv), bb, v.x, out}, NoFin{}, stop, 2);
            else
                spmv<T, 0>(Lv.A, avals<T>(Lv.A), GPlain<T, NB>{v.x},
                           EPost<T, NB, false>{dl1inv<T>(Lv), bb, v.x, out}, NoFin{}, stop);
        }
        AMG_HIP(hipGetLastError());
    }

    // ---------------- graph capture ----------------
    // Records the launches of body() on the private capture stream and
    // instantiates them; the graph is replayed on the context's stream.
    template <class F> hipGraphExec_t capture(F &&body) {
        const hipStream_t saved = s;
        s = c.cap_stream;
        AMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipGraph_t g = nullptr;
        try {
            body();
        } catch (...) {
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            s = saved;
            throw;
        }
        AMG_HIP(hipStreamEndCapture(s, &g));
        s = saved;
        hipGraphExec_t e = nullptr;
        const hipError_t rc = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        AMG_HIP(rc);
        c.graphs.push_back(e);
        return e;
    }

    void launch(hipGraphExec_t g) { AMG_HIP(hipGraphLaunch(g, s)); }

    // The finalize kernels write each CG's mailbox in pinned host memory; an
    // event marks how far the stream has run, so no copy is enqueued.
    void post_flag(int slot) { AMG_HIP(hipEventRecord(pev[slot], s)); }

    template <typename T> bool wait_flag(int slot, const CgWs<T> &w) {
        AMG_HIP(hipEventSynchronize(pev[slot]));
        return __atomic_load_n(&w.hmail->all_conv, __ATOMIC_ACQUIRE) != 0;
    }

    // ---------------- conjugate gradients ----------------
    // JAC: Jacobi preconditioner (mass matrices), else the V-cycle from level j.
    // One CG iteration (p_new = z + beta p_old, q = A p_new, alpha; x, r update
    // and the convergence test; z = B r and beta) is a fixed sequence of
    // launches on fixed buffers, captured once per workspace in two graphs
    // (even and odd iterations swap p_old and p_new).  The host launches the
    // iterations it expects from the previous solve at this level, then keeps
    // one iteration in flight while it reads the convergence flag of the one
    // before; iterations after convergence return at once in every kernel.
    // Returns the largest iteration count over the columns; x_out gets x.
    // MIX (FP64 CG only): the preconditioner is the float32 V-cycle; the CG
    // update also writes r in float32 and the next direction reads z from it.
    template <typename T, bool JAC, bool MIX = false>
    void cg_iter(int j, const DCsr &A, const T *vals, const T *dinv, CgWs<T> &w, T *pold, T *pnew) {
        const int n = A.n;
        const int *stop = &w.sc->all_conv;
        const int fused = w.fused;
        const FusedFin<NB, JAC> pro{w.sc, part[1], pgrid[1], part[2], pgrid[2]};
        // the first kernel: (fused: the previous finalize,) p = z + beta pold, q = A p, p.q partials
        auto first = [&](auto gx, auto ep) {
            if (fused) spmv<T, 1>(A, vals, gx, ep, NoFin{}, stop, 0, pro);
            else spmv<T, 1>(A, vals, gx, ep, NoFin{}, stop, 0);
        };
        if constexpr (MIX) {
            static_assert(std::is_same_v<T, double> && !JAC, "float32 preconditioning of the FP64 CG only");
            float *r32 = c.ws[j].b32, *z32 = c.ws[j].d32;
            first(GZ<T, NB, float>{z32}, ECgQR<T, NB, float>{z32, pold, pnew, w.q, w.sc});
            cg_update<T, false>(n, nullptr, w.r, nullptr, pnew, w.q, nullptr, w.sc, 0, stop, r32,
                                vcws<float>(c.ws[j]).x, c.lev[j].dl1inv32, first_scale(), fused);
            vcycle<float>(j, r32, z32, true, stop);
            if (!fused)
                hipLaunchKernelGGL((fin2_kernel<NB, FinUB<NB>>), dim3(1), dim3(kFinBlock), 0, s, part[1],
                                   pgrid[1], part[2], pgrid[2], FinUB<NB>{w.sc}, stop);
            return;
        }
        first(GZ<T, NB>{w.z}, ECgQR<T, NB>{w.z, pold, pnew, w.q, w.sc});
        if constexpr (JAC)
            cg_update<T, JAC>(n, nullptr, w.r, w.z, pnew, w.q, dinv, w.sc, 0, stop, nullptr, nullptr, nullptr, 1.0,
                              fused);
        else
            cg_update<T, JAC>(n, nullptr, w.r, vcws<T>(c.ws[j]).x, pnew, w.q, dl1inv<T>(c.lev[j]), w.sc, 0, stop,
                              nullptr, nullptr, nullptr, first_scale(), fused);
        if constexpr (JAC) {
            if (!fused) finish<2>(1, FinUpd<NB, true>{w.sc}, stop);
        } else {
            vcycle<T>(j, w.r, w.z, true, stop);
            if (!fused)
                hipLaunchKernelGGL((fin2_kernel<NB, FinUB<NB>>), dim3(1), dim3(kFinBlock), 0, s, part[1],
                                   pgrid[1], part[2], pgrid[2], FinUB<NB>{w.sc}, stop);
        }
    }

    // fused mode: the finalize of the last update when the iteration limit ends the loop
    template <bool JAC> void fused_tail(CgWs<double> &w) { fused_tail_impl<JAC>(w.sc); }
    template <bool JAC> void fused_tail(CgWs<float> &w) { fused_tail_impl<JAC>(w.sc); }
    template <bool JAC> void fused_tail_impl(CgScal *sc) {
        if constexpr (JAC)
            hipLaunchKernelGGL((fin_kernel<2, NB, FinFusedTail<NB, true>>), dim3(1), dim3(kFinBlock), 0, s, part[1],
                               pgrid[1], FinFusedTail<NB, true>{sc}, &sc->all_conv);
        else
            hipLaunchKernelGGL((fin2_kernel<NB, FinFusedTail<NB, false>>), dim3(1), dim3(kFinBlock), 0, s,
                               part[1], pgrid[1], part[2], pgrid[2], FinFusedTail<NB, false>{sc},
                               &sc->all_conv);
    }

    // phase 0: the whole solve; 1: start only (initialisation and the first
    // batch, margin more iterations than the previous solve needed, no wait
    // for the device); 2: finish a started solve (the polling loop from where
    // phase 1 left it, on the same solver's stream)
    template <typename T, bool JAC, bool MIX = false>
    int cg(int j, const DCsr &A, const T *vals, const double *mdinv, CgWs<T> &w, const T *b, T *x, double rtol,
           int maxit, int nlive, int phase = 0, int margin = 0) {
        const int n = A.n;
        const int *stop = &w.sc->all_conv;
        const T *dinv = nullptr;
        if constexpr (JAC) dinv = mdinv;
        float *r32 = nullptr, *x32 = nullptr;
        const float *d32 = nullptr;
        T *z0 = w.z;
        const T *d0 = dinv;
        if constexpr (MIX) {
            r32 = c.ws[j].b32;
            x32 = vcws<float>(c.ws[j]).x;
            d32 = c.lev[j].dl1inv32;
            z0 = nullptr;
        } else if constexpr (!JAC) {
            z0 = vcws<T>(c.ws[j]).x;
            d0 = dl1inv<T>(c.lev[j]);
        }
        if (w.fused < 0) {
            // fold each finalize into the next iteration's first kernel when every
            // workgroup can afford to sum the partials it needs
            long q = (JAC ? 2L : 1L) * grid_rows((long)n * NB, kBlock, red_grid_max<NB>()) * NB;
            if constexpr (!JAC) q += (long)red_grid<std::conditional_t<MIX, float, T>>(A) * NB;
            w.fused = q <= kFusedPartials ? 1 : 0;
        }
        const int fused = w.fused;
        if (phase != 2)
            elem<JAC ? 2 : 1>(n, OpInit<T, NB, JAC>{b, w.r, x, w.p0, z0, d0, r32, x32, d32, first_scale()},
                              FinInit<NB, JAC>{w.sc, rtol, nlive, (void *)x, fused}, nullptr, fused ? 1 : 0);
        // captured graphs for every CG (1) or only for the mass-matrix CGs (2),
        // whose two-kernel iterations outrun eager launches from the host
        const bool graphs = c.o.use_graphs == 1 || (c.o.use_graphs == 2 && JAC);
        auto first_precond = [&] {
            if constexpr (MIX) vcycle<float>(j, c.ws[j].b32, c.ws[j].d32, true, stop);
            else vcycle<T>(j, w.r, w.z, true, stop);
            if (!fused) finish<1>(2, FinRho0<NB>{w.sc}, stop);
        };
        // Iterations go out in pairs (p0 -> p1 -> p0), one graph launch per pair,
        // so the iteration count before a launch is even; a single iteration is
        // issued only as the last one before maxit.  Iterations past convergence
        // return at once in every kernel.
        if (graphs && !w.g2) {
            if constexpr (!JAC) w.g0 = capture(first_precond);
            w.g2 = capture([&] {
                cg_iter<T, JAC, MIX>(j, A, vals, dinv, w, w.p0, w.p1);
                cg_iter<T, JAC, MIX>(j, A, vals, dinv, w, w.p1, w.p0);
            });
            // a mass iteration is two small kernels, faster than the host issues
            // one launch per iteration: its first batch goes out eight at a time
            if constexpr (JAC)
                w.g8 = capture([&] {
                    for (int k = 0; k < 8; k += 2) {
                        cg_iter<T, JAC, MIX>(j, A, vals, dinv, w, w.p0, w.p1);
                        cg_iter<T, JAC, MIX>(j, A, vals, dinv, w, w.p1, w.p0);
                    }
                });
        }
        if constexpr (!JAC) {
            if (phase != 2) {
                if (graphs) launch(w.g0);
                else first_precond();
            }
        }
        int it = phase == 2 ? w.run_it : 0;
        auto step = [&]() {
            const bool pair = maxit - it >= 2;
            if (graphs) {
                if (!pair && !w.ga) w.ga = capture([&] { cg_iter<T, JAC, MIX>(j, A, vals, dinv, w, w.p0, w.p1); });
                launch(pair ? w.g2 : w.ga);
            } else {
                cg_iter<T, JAC, MIX>(j, A, vals, dinv, w, w.p0, w.p1);
                if (pair) cg_iter<T, JAC, MIX>(j, A, vals, dinv, w, w.p1, w.p0);
            }
            it += pair ? 2 : 1;
        };
        // The iterations the previous solve at this level needed (one more when
        // fused: the convergence of update k is decided in iteration k + 1) go
        // out at once, and the host waits for them: usually they suffice, and
        // nothing runs past convergence.  When they do not, the host keeps two
        // launches in flight beyond the last one it has seen (it waits on the
        // older one's event while the newer one runs), reading the mailbox
        // after each event; at most one launch then runs past convergence,
        // returning at once in every kernel.
        constexpr int kRing = Ctx::kPollRing;
        int posted = 1, seen = 0;
        if (phase != 2) {
            const int first = std::min(std::max(1, w.pred + (fused ? 1 : 0) + margin), maxit);
            while (it < first) {
                if (graphs && w.g8 && first - it >= 8) {
                    launch(w.g8);
                    it += 8;
                } else {
                    step();
                }
            }
            post_flag(0);
            if (phase == 1) {
                w.run_it = it;
                return 0;
            }
        }
        bool done = false;
        while (!done) {
            if (it >= maxit) {
                if (fused) fused_tail<JAC>(w);
                post_flag(posted % kRing);
                ++posted;
                AMG_HIP(hipEventSynchronize(pev[(posted - 1) % kRing]));
                done = __atomic_load_n(&w.hmail->all_conv, __ATOMIC_ACQUIRE) != 0;
                break;
            }
            if (posted - seen < (seen == 0 ? 1 : 2)) {
                step();
                post_flag(posted % kRing);
                ++posted;
                continue;
            }
            done = wait_flag(seen % kRing, w);
            ++seen;
        }
        // the last posted event covers every launch: the mailbox is final
        AMG_HIP(hipEventSynchronize(pev[(posted - 1) % kRing]));
        const Mail &m = *w.hmail;
        if (!m.all_conv) {
            w.pred = it;
            fail(AMG_ERR_NOCONV, std::string(JAC ? "mass" : "inner") + " CG did not converge at level " +
                                     std::to_string(j));
        }
        if (m.bad)
            fail(AMG_ERR_NOCONV, std::string(JAC ? "mass" : "inner") + " CG breakdown at level " + std::to_string(j));
        w.pred = std::max(0, m.iters);  // fused: -1 when every column stopped before the first update
        return w.pred;
    }

    // ---------------- solves with A_j ----------------
    void solve_A(int j, const double *f, double *x, double rtol) {
        if (j == c.L - 1 || c.lev[j].Ainv) {
            dense_apply<double>(j == c.L - 1 ? c.dAc : c.lev[j].dA, f, x, nullptr);
            AMG_HIP(hipGetLastError());
            return;
        }
        if (c.o.inner_precision == 32 && c.o.mixed_mode == 1) {
            solve_A_mixed(j, f, x, rtol);
            return;
        }
        Level &L = c.lev[j];
        const int it = c.o.inner_precision == 32
                           ? cg<double, false, true>(j, L.A, L.A.v, nullptr, c.ws[j].inmx, f, x, rtol,
                                                     c.o.inner_maxit, NB)
                           : cg<double, false>(j, L.A, L.A.v, nullptr, c.ws[j].in64, f, x, rtol, c.o.inner_maxit, NB);
        c.st.inner_solves++;
        c.st.inner_iters += it;
        c.st.inner_max = std::max<long>(c.st.inner_max, it);
    }

    // FP64 iterative refinement around the float32 CG:
    //   s = ||r||, d = CG32(fp32(r / s)), x += s d, r = f - A x (FP64),
    // until ||r|| <= rtol ||f|| per column.
    void solve_A_mixed(int j, const double *f, double *x, double rtol) {
        Level &L = c.lev[j];
        LevelWs &w = c.ws[j];
        const int n = L.n;
        elem<1>(n, OpCopyNorm<NB>{f, w.rr, x}, FinRefInit<NB>{c.rsd, rtol, NB}, nullptr);
        wait_mail();
        int steps = 0;
        while (c.rmail->nlive > 0) {
            if (steps >= c.o.refine_maxit) fail(AMG_ERR_NOCONV, "refinement did not converge");
            elem<0>(n, OpCastScale<NB>{w.b32, w.rr, c.rsd}, NoFin{}, nullptr);
            const int it = cg<float, false>(j, L.A, L.A.v32, nullptr, w.in32, w.b32, w.d32, c.o.inner32_rtol,
                                            c.o.inner_maxit, NB);
            c.st.inner_iters += it;
            c.st.inner_max = std::max<long>(c.st.inner_max, it);
            elem<0>(n, OpRefAdd<NB>{x, w.d32, c.rsd}, NoFin{}, nullptr);
            spmv<double, 1>(L.A, L.A.v, GPlain<double, NB>{x}, EResid<NB>{f, w.rr}, FinRefine<NB>{c.rsd}, nullptr);
            wait_mail();
            ++steps;
            c.st.refine++;
            if (c.rmail->stagnated) fail(AMG_ERR_NOCONV, "refinement stagnated at level " + std::to_string(j));
        }
        c.st.inner_solves++;
    }

    void mass_solve(int j, const double *b, double *x) {
        Level &L = c.lev[j];
        if (L.Minv) {
            dense_apply<double>(L.dM, b, x, nullptr);
            AMG_HIP(hipGetLastError());
            return;
        }
        const int it =
            cg<double, true>(j, L.M, L.M.v, L.mdinv, c.ws[j].mass, b, x, c.o.mass_rtol, c.o.mass_maxit, NB);
        c.st.mass_iters += it;
    }

    // An iterative mass solve split in two on this (side) solver, in its own
    // workspace: mass_start enqueues the initialisation and two more iterations
    // than the previous such solve needed, without waiting; mass_finish
    // iterates on until the mailbox reports convergence (usually it already
    // has), so x is final once it returns and this stream has run.
    void mass_start(int j, const double *b, double *x) {
        Level &L = c.lev[j];
        cg<double, true>(j, L.M, L.M.v, L.mdinv, c.ws[j].mass2, b, x, c.o.mass_rtol, c.o.mass_maxit, NB, 1, 2);
    }
    void mass_finish(int j, const double *b, double *x) {
        Level &L = c.lev[j];
        c.st.mass_iters +=
            cg<double, true>(j, L.M, L.M.v, L.mdinv, c.ws[j].mass2, b, x, c.o.mass_rtol, c.o.mass_maxit, NB, 2);
    }

    // y = M_which x at level j (0: M_u, 1: M_y = DMD, 2: M_yu = DM, 3: M_yu^T = MD);
    // with dotx, dots[c] = dotx_c . y_c (device)
    void mass_apply(int j, int which, const double *x, double *y, const double *dotx, double *dots) {
        Level &L = c.lev[j];
        const uint8_t *mk = (j == 0 && c.has_mask) ? c.mask0 : nullptr;
        const uint8_t *gm = (which == 1 || which == 3) ? mk : nullptr;
        const uint8_t *em = (which == 1 || which == 2) ? mk : nullptr;
        if (dotx)
            spmv<double, 1>(L.M, L.M.v, GLin<NB>{x, gm, nullptr, 0.0},
                            ELin<NB>{y, em, 1.0, nullptr, 0.0, nullptr, 0.0, dotx}, FinStore<NB>{dots}, nullptr);
        else
            spmv<double, 0>(L.M, L.M.v, GLin<NB>{x, gm, nullptr, 0.0},
                            ELin<NB>{y, em, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr}, NoFin{}, nullptr);
        AMG_HIP(hipGetLastError());
    }

    // y = K_j u = A_j^{-1} M_yu u
    void state_solve(int j, const double *u, double *y, double rtol) {
        LevelWs &w = c.ws[j];
        mass_apply(j, 2, u, w.hf, nullptr, nullptr);
        solve_A(j, w.hf, y, rtol);
    }

    // z = K_j^T w = M_yu^T A_j^{-1} w
    void adjoint_solve(int j, const double *wv, double *z, double rtol) {
        LevelWs &w = c.ws[j];
        solve_A(j, wv, w.ht, rtol);
        mass_apply(j, 3, w.ht, z, nullptr, nullptr);
    }

    // Hu = K^T M_y K u + beta M_u u, formed as M (D t + beta u) with
    // t = A^{-1} M_y A^{-1} M_yu u; with rminus, Hu = rminus - H u.
    void hessian_apply(int j, const double *u, double *Hu, double rtol, const double *rminus) {
        Range rg(j == 0 ? "hessian_apply" : "hessian_apply_coarse");
        Level &L = c.lev[j];
        LevelWs &w = c.ws[j];
        const uint8_t *mk = (j == 0 && c.has_mask) ? c.mask0 : nullptr;
        mass_apply(j, 2, u, w.hf, nullptr, nullptr);
        solve_A(j, w.hf, w.hy, rtol);
        mass_apply(j, 1, w.hy, w.hw, nullptr, nullptr);
        solve_A(j, w.hw, w.ht, rtol);
        spmv<double, 0>(L.M, L.M.v, GLin<NB>{w.ht, mk, u, c.o.beta},
                        ELin<NB>{Hu, nullptr, rminus ? -1.0 : 1.0, rminus, 1.0, nullptr, 0.0, nullptr}, NoFin{},
                        nullptr);
        AMG_HIP(hipGetLastError());
    }

    // ---------------- multilevel preconditioner (practical form) ----------------
    // C_l(r) = S_l (B_{l+1} q - beta^{-1} M_{l+1}^{-1} q) + beta^{-1} M_l^{-1} r (+ zprev),
    // q = S_l^T r
    // mself: M_l^{-1} r when the caller has it already (the parent C_{l-1}
    // formed M_l^{-1} (S_{l-1}^T r) for its own correction term), else null
    void Cop(int l, const double *r, double *out, const double *zprev, const double *mself = nullptr) {
        Level &Lv = c.lev[l];
        LevelWs &w1 = c.ws[l + 1];
        LevelWs &w0 = c.ws[l];
        // M_l^{-1} r does not depend on the coarser work below: an iterative one
        // runs on the side stream meanwhile (one such solve at a time)
        const bool side = !mself && !Lv.Minv && !c.side_busy;
        Solver<NB> S2(c, c.side, c.part2, c.pgrid2, c.poll_ev2);
        struct Busy {  // released on every way out (the side solve writes only its own buffers)
            bool &b;
            bool on;
            ~Busy() {
                if (on) b = false;
            }
        } busy{c.side_busy, side};
        if (side) {
            c.side_busy = true;
            AMG_HIP(hipEventRecord(c.mass_ev[0], s));
            AMG_HIP(hipStreamWaitEvent(c.side, c.mass_ev[0], 0));
            S2.mass_start(l, r, w0.ml_mself);
        }
        spmv<double, 0>(Lv.St, Lv.St.v, GPlain<double, NB>{r}, EStore<double, NB>{w1.ml_in}, NoFin{}, nullptr);
        mass_solve(l + 1, w1.ml_in, w1.ml_mup);
        Bop(l + 1, w1.ml_in, w1.ml_out);
        if (side) {
            S2.mass_finish(l, r, w0.ml_mself);
            AMG_HIP(hipEventRecord(c.mass_ev[1], c.side));
            AMG_HIP(hipStreamWaitEvent(s, c.mass_ev[1], 0));
            mself = w0.ml_mself;
        } else if (!mself) {
            mass_solve(l, r, w0.ml_mself);
            mself = w0.ml_mself;
        }
        const double ib = 1.0 / c.o.beta;
        spmv<double, 0>(Lv.S, Lv.S.v, GLin<NB>{w1.ml_out, nullptr, w1.ml_mup, -ib},
                        ELin<NB>{out, nullptr, 1.0, mself, ib, zprev, 1.0, nullptr}, NoFin{}, nullptr);
        AMG_HIP(hipGetLastError());
    }

    // B_{ell-1} = H_{ell-1}^{-1} (dense); B_l = 2 C_l - C_l H_l C_l as the two
    // calls of Algorithm MLAS (0 < l < ell-1); B_0 = C_0
    void Bop(int l, const double *r, double *z) {
        if (l == c.ell - 1) {
            if (c.Hinv) {
                dense_apply<double>(c.dH, r, z, nullptr);
                AMG_HIP(hipGetLastError());
            } else {
                hess_cg(l, r, z);
            }
            return;
        }
        if (l == 0) {
            Cop(0, r, z, nullptr);
            return;
        }
        // B_l is only reached from C_{l-1}, which left M_l^{-1} r in ml_mup of this level
        LevelWs &w = c.ws[l];
        Cop(l, r, w.ml_z1, nullptr, w.ml_mup);
        hessian_apply(l, w.ml_z1, w.ml_t, c.o.precond_inner_rtol, r);  // t = r - H_l z1
        // the second C_l's mass solve from the first's: at l >= 1 every mass
        // matrix is M_l, so H_l z1 = M_l (ht + beta z1) (ht the Hessian's inner
        // result) and M_l^{-1} t = M_l^{-1} r - (ht + beta z1)
        elem<0>(c.lev[l].n, OpSubSum<NB>{w.ml_mself, w.ml_mup, w.ht, w.ml_z1, c.o.beta}, NoFin{}, nullptr);
        Cop(l, w.ml_t, z, w.ml_z1, w.ml_mself);                         // z = z1 + C_l t
    }

    // Coarsest Hessian level too large to invert densely: CG on G_l in the
    // L^2 inner product to coarse_hess_rtol from x = 0 (Section 5.2), i.e. CG on
    // H_l = M_l G_l preconditioned by M_l^{-1}, stopped when
    // r.M^{-1}r <= rtol^2 b.M^{-1}b (the relative M-norm of G_l x - g).
    void hess_cg(int l, const double *b, double *x) {
        Range rg("coarse_hessian_cg");
        const int n = c.lev[l].n;
        CgWs<double> &w = c.ws[l].hcg;
        elem<0>(n, OpAxpby<NB>{w.r, b, nullptr, 1.0, 0.0}, NoFin{}, nullptr);
        elem<0>(n, OpAxpby<NB>{x, b, nullptr, 0.0, 0.0}, NoFin{}, nullptr);
        mass_solve(l, w.r, w.z);
        elem<0>(n, OpAxpby<NB>{w.p0, w.z, nullptr, 1.0, 0.0}, NoFin{}, nullptr);
        elem<2>(n, OpDot<NB>{b, w.z, w.r, w.z}, FinOuterInit<NB>{w.sc, c.o.coarse_hess_rtol, NB}, nullptr);
        elem<1>(n, OpDot<NB>{w.r, w.z, nullptr, nullptr}, FinRho<NB>{w.sc}, nullptr);
        read_sc(w.sc);
        for (int it = 0; !c.hsc->all_conv; ++it) {
            if (it >= c.o.outer_maxit) fail(AMG_ERR_NOCONV, "coarsest-level Hessian CG did not converge");
            hessian_apply(l, w.p0, w.q, c.o.precond_inner_rtol, nullptr);
            elem<1>(n, OpDot<NB>{w.p0, w.q, nullptr, nullptr}, NoFin{}, nullptr, 0);
            cg_update<double, false>(n, x, w.r, nullptr, w.p0, w.q, nullptr, w.sc, 0, nullptr);
            mass_solve(l, w.r, w.z);
            elem<1>(n, OpDot<NB>{w.r, w.z, nullptr, nullptr}, FinRzConv<NB>{w.sc}, nullptr);
            read_sc(w.sc);
            for (int col = 0; col < NB; ++col)
                if (c.hsc->s[col].bad) fail(AMG_ERR_NOCONV, "coarsest-level Hessian CG breakdown");
            if (c.hsc->all_conv) break;
            elem<0>(n, OpPUpd<NB>{w.p0, w.z, w.sc}, NoFin{}, nullptr);
        }
        c.st.coarse_cg += 1;
    }

    void precond(const double *r, double *z) {
        Range rg("hessian_precond_apply");
        if (c.o.precond) Bop(0, r, z);
        else elem<0>(c.N, OpAxpby<NB>{z, r, nullptr, 1.0, 0.0}, NoFin{}, nullptr);
    }

    // ---------------- outer CG on H_0 (Section 5.3) ----------------
    int outer(const double *b, double *x, bool have_x0, double rtol, int nlive, int *iters_out) {
        const int n = c.N;
        CgWs<double> &w = c.outer;
        int total = 0;  // iterations over all attempts
        for (;;) {
            if (have_x0) {
                c.ph.mark(kPhHess, s);
                hessian_apply(0, x, w.r, c.o.inner_rtol, b);  // r = b - H x0
                c.ph.mark(kPhOuter, s);
            } else {
                elem<0>(n, OpAxpby<NB>{w.r, b, nullptr, 1.0, 0.0}, NoFin{}, nullptr);
                elem<0>(n, OpAxpby<NB>{x, b, nullptr, 0.0, 0.0}, NoFin{}, nullptr);
            }
            elem<2>(n, OpDot<NB>{b, b, w.r, w.r}, FinOuterInit<NB>{w.sc, rtol, nlive}, nullptr);
            c.ph.mark(kPhPrec, s);
            precond(w.r, w.z);
            c.ph.mark(kPhOuter, s);
            elem<1>(n, OpDot<NB>{w.r, w.z, nullptr, nullptr}, FinRho<NB>{w.sc}, nullptr);
            elem<0>(n, OpAxpby<NB>{w.p0, w.z, nullptr, 1.0, 0.0}, NoFin{}, nullptr);
            read_sc(w.sc);
            int it = 0;
            bool indefinite = c.hsc->indefinite;
            bool done = c.hsc->all_conv;
            while (!done && !indefinite) {
                if (it >= c.o.outer_maxit) {
                    *iters_out = total + it;
                    return AMG_ERR_NOCONV;
                }
                Range rg("outer_iteration");
                c.ph.mark(kPhHess, s);
                hessian_apply(0, w.p0, w.q, c.o.inner_rtol, nullptr);
                c.ph.mark(kPhOuter, s);
                elem<1>(n, OpDot<NB>{w.p0, w.q, nullptr, nullptr}, NoFin{}, nullptr, 0);
                cg_update<double, false>(n, x, w.r, nullptr, w.p0, w.q, nullptr, w.sc, 1, nullptr);
                finish<1>(1, FinUpd<NB, false>{w.sc}, nullptr);
                ++it;
                read_sc(w.sc);
                if (c.hsc->indefinite) {
                    indefinite = true;
                    break;
                }
                if (c.hsc->all_conv) break;
                c.ph.mark(kPhPrec, s);
                precond(w.r, w.z);
                c.ph.mark(kPhOuter, s);
                elem<1>(n, OpDot<NB>{w.r, w.z, nullptr, nullptr}, FinBeta<NB>{w.sc, 1}, nullptr);
                elem<0>(n, OpPUpd<NB>{w.p0, w.z, w.sc}, NoFin{}, nullptr);
            }
            total += it;
            if (!indefinite) {
                *iters_out = total;
                return AMG_OK;
            }
            if (!(c.o.auto_levels && c.ell > 1)) {
                *iters_out = total;
                return AMG_ERR_INDEFINITE;
            }
            // one Hessian level fewer, and CG again from the last iterate: every
            // step taken had p.q > 0, so it is no worse than zero (a column that
            // met p.q <= 0 was not updated by that step)
            form_dense_hessian(c, c.ell - 1);
            have_x0 = true;
        }
    }
};

}  // namespace amg
