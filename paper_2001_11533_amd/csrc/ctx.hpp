// The library context: the AMG hierarchy, dense coarse data and all solve
// workspaces, sized once at setup for the widest batch.
#pragma once

#include <memory>
#include <type_traits>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace amg {

// A dense coarse operator for x = Inv b: row-major with the row stride ld
// padded to a multiple of 64 entries (zeros), in FP64 and float32.
struct DenseOp {
    int n = 0, ld = 0;
    double *m64 = nullptr;
    float *m32 = nullptr;
};

struct Level {
    int n = 0;
    DCsr A, S, St, M;           // A_j, S_j (n_j x n_{j+1}), S_j^T, mass M_j
    DCsr T;                     // A_j S_j (level < L-1; its pattern contains that of S_j)
    double *Ts = nullptr;       // S_j's values on T's pattern (zero where S_j has no entry)
    float *Ts32 = nullptr;
    uint16_t *Tc16 = nullptr;   // T's columns as 16-bit values (when n_{j+1} <= 65536)
    double *dl1inv = nullptr;   // 1 / sum_k |a_ik|
    float *dl1inv32 = nullptr;
    double *mdinv = nullptr;    // 1 / diag(M_j)
    int *agg = nullptr;         // level < L-1
    uint8_t *root = nullptr;
    const uint8_t *mask = nullptr;  // Dirichlet flags, level 0 only
    double *Ainv = nullptr;     // small coarse levels: dense inverses of A_j and M_j
    double *Minv = nullptr;
    DenseOp dA, dM;             // their padded apply copies
};

template <typename T> struct CgWs {
    T *x = nullptr, *r = nullptr, *z = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    CgScal *sc = nullptr;
    Mail *hmail = nullptr;  // host view of the mailbox the finalize kernels write
    int pred = 0;  // iteration count of the previous solve (poll schedule)
    int run_it = 0; // iterations launched by a started (phase 1) solve
    int fused = -1; // 1: each iteration's finalize runs in the next iteration's first kernel
    // captured graphs: first preconditioner application, iteration p0->p1 (a
    // last single step only), the pair p0->p1->p0
    hipGraphExec_t g0 = nullptr, ga = nullptr, g2 = nullptr;
    hipGraphExec_t g8 = nullptr;  // Jacobi CG: eight iterations (four pairs) in one launch
};

template <typename T> struct VcWs {
    T *b = nullptr, *x = nullptr, *r = nullptr, *x2 = nullptr;
    T *t = nullptr;  // Chebyshev smoothing: the iterate after pre-smoothing
};

struct LevelWs {
    CgWs<double> in64, mass, hcg;  // inner A-solves, mass solves, coarsest-Hessian CG
    CgWs<double> mass2;            // mass solves run on the side stream
    CgWs<double> inmx;             // inner A-solves preconditioned by the float32 V-cycle
    CgWs<float> in32;
    VcWs<double> vc64;
    VcWs<float> vc32;
    // mixed refinement
    double *rx = nullptr, *rr = nullptr;
    float *b32 = nullptr, *d32 = nullptr;
    // Hessian apply temporaries
    double *hf = nullptr, *hy = nullptr, *hw = nullptr, *ht = nullptr;
    // multilevel preconditioner
    double *ml_in = nullptr, *ml_out = nullptr, *ml_mup = nullptr, *ml_mself = nullptr;
    double *ml_z1 = nullptr, *ml_t = nullptr;
};

struct Stats {
    long inner_solves = 0, inner_iters = 0, inner_max = 0, mass_iters = 0, refine = 0, coarse_cg = 0;
    double bytes = 0.0;  // algorithmic bytes of the sparse and dense products issued
    void reset() { *this = Stats(); }
};

// Phases of a reduced solve whose device time amg_info reports.
enum Phase { kPhRhs = 0, kPhHess = 1, kPhPrec = 2, kPhOuter = 3, kPhTrue = 4, kPhEnd = -1 };

// Device time per phase of one call: an event is recorded on the main stream
// where one phase ends and the next begins (work of the side streams joins the
// main stream before it is used, so it falls inside the phase that waits for
// it); the elapsed times are summed per phase once the call's work has run.
struct PhaseTimer {
    std::vector<hipEvent_t> ev;
    std::vector<int> lab;
    int used = 0;
    bool on = false;
    void start() {
        used = 0;
        on = true;
    }
    void mark(int phase, hipStream_t s) {
        if (!on) return;
        if (used == (int)ev.size()) {
            hipEvent_t e = nullptr;
            AMG_HIP(hipEventCreate(&e));
            ev.push_back(e);
            lab.push_back(kPhEnd);
        }
        AMG_HIP(hipEventRecord(ev[used], s));
        lab[used++] = phase;
    }
    // after the stream has run past the last mark
    void sum(double (&ms)[8]) {
        for (int k = 0; k + 1 < used; ++k) {
            float t = 0.f;
            AMG_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
            if (lab[k] >= 0 && lab[k] < 8) ms[lab[k]] += t;
        }
        on = false;
    }
    void destroy() {
        for (auto e : ev) (void)hipEventDestroy(e);
        ev.clear();
        lab.clear();
    }
};

struct Ctx {
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream used only to capture graphs
    hipStream_t side = nullptr;         // setup work that overlaps the main stream (dense inverses)
    hipStream_t gal = nullptr;          // setup: the mass matrices' Galerkin products beside the stiffness ones
    hipEvent_t gal_ev[2] = {nullptr, nullptr};
    int *iscratch2 = nullptr;           // scratch words of the products on gal (device, pinned host)
    int *hiscr2 = nullptr;
    hipEvent_t side_ev[2] = {nullptr, nullptr};  // fork and join of the side stream
    std::vector<hipGraphExec_t> graphs; // every instantiated graph (freed with the context)
    static constexpr int kPollRing = 4;
    hipEvent_t poll_ev[kPollRing] = {nullptr, nullptr, nullptr, nullptr};
    // solve phase: a mass solve on the side stream beside the main work, with
    // its own reduction partials and polling events; its fork and join events
    double *part2[3] = {nullptr, nullptr, nullptr};
    int pgrid2[3] = {0, 0, 0};
    hipEvent_t poll_ev2[kPollRing] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t mass_ev[2] = {nullptr, nullptr};
    bool side_busy = false;
    amg_opts o{};
    Arena arena;
    int N = 0;
    int L = 0, ell = 0;
    int nbp = 1;  // padded batch width of the workspaces
    std::vector<Level> lev;
    std::vector<LevelWs> ws;
    // dense coarse data
    double *Ainv = nullptr;  // inverse of A_{L-1}, row-major
    int nAinv = 0;
    double *Hdense = nullptr, *Hinv = nullptr;  // practical-form Hessian at level ell-1
    int nH = 0;
    DenseOp dAc, dH;  // padded apply copies of Ainv and Hinv
    // reductions (one stream: a single partial buffer and ticket suffice)
    double *part[3] = {nullptr, nullptr, nullptr};  // reduction partials [2*16*kMaxGrid] each
    int pgrid[3] = {0, 0, 0};                       // workgroups that wrote each buffer
    double *dscratch = nullptr;  // small device scalars [64]
    int *iscratch = nullptr;     // small device ints [64]
    // host mirrors
    CgScal *hsc = nullptr;       // pinned
    double *hscr = nullptr;      // pinned [64]
    int *hiscr = nullptr;        // pinned [64]
    // outer CG workspace (level 0)
    CgWs<double> outer;
    // CG scalars used only by kernel timing (amg_time_kernel), and their mailbox
    CgScal *tsc = nullptr;
    Mail *tsc_mail = nullptr;
    double *ox = nullptr, *ob = nullptr, *obq = nullptr;
    double *pk_in = nullptr, *pk_out = nullptr;  // packing buffers [N x nbp]
    // refinement per-column data (device) and its pinned host mirror
    RefScal *rsd = nullptr;
    Mail *rmail = nullptr;              // host view of the refinement mailbox
    Mail *mails = nullptr;              // pinned pool of mailboxes
    int nmail = 0;
    Stats st;
    PhaseTimer ph;
    std::string err;
    bool has_mask = false;
    uint8_t *mask0 = nullptr;
};

// setup.hip
void build_hierarchy(Ctx &c, const amg_csr &A, const amg_csr &M, const uint8_t *dirichlet);
void form_dense_hessian(Ctx &c, int ell);

template <typename T> inline const T *avals(const DCsr &A) {
    if constexpr (std::is_same_v<T, double>) return A.v;
    else return A.v32;
}
template <typename T> inline const T *tsvals(const Level &L) {
    if constexpr (std::is_same_v<T, float>) return L.Ts32;
    else return L.Ts;
}
template <typename T> inline const T *dl1inv(const Level &L) {
    if constexpr (std::is_same_v<T, double>) return L.dl1inv;
    else return L.dl1inv32;
}
template <typename T> inline VcWs<T> &vcws(LevelWs &w) {
    if constexpr (std::is_same_v<T, double>) return w.vc64;
    else return w.vc32;
}

}  // namespace amg
