// C ABI of the library (declared in include/amghess.h).  Every entry point
// catches internal errors and returns a status code.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "solver.hpp"

namespace amg {
namespace {

thread_local std::string g_setup_err;

int pad_nb(int nb) { return nb <= 1 ? 1 : nb <= 2 ? 2 : nb <= 4 ? 4 : nb <= 8 ? 8 : 16; }

template <class F> int dispatch_nb(int nbp, F &&f) {
    switch (nbp) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 8: return f(std::integral_constant<int, 8>{});
        default: return f(std::integral_constant<int, 16>{});
    }
}

template <class F> int guarded(Ctx *c, F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        if (c) c->err = e.msg;
        else g_setup_err = e.msg;
        (void)hipGetLastError();
        return e.code;
    } catch (const std::exception &e) {
        if (c) c->err = e.what();
        else g_setup_err = e.what();
        return AMG_ERR_HIP;
    }
}

// a mailbox from the pinned pool (zeroed) and its device view
Mail *take_mail(Ctx &c, Mail **dev_view) {
    if (c.nmail >= 64) fail(AMG_ERR_OOM, "mailbox pool exhausted");
    Mail *h = &c.mails[c.nmail++];
    std::memset(h, 0, sizeof(Mail));
    void *d = nullptr;
    AMG_HIP(hipHostGetDevicePointer(&d, h, 0));
    *dev_view = static_cast<Mail *>(d);
    return h;
}

// The scalar blocks of all CG workspaces sit in one device array that a single
// copy initialises (zeroed, each with its mailbox's device view): one transfer
// instead of a blocking memset and copy per workspace.
struct ScalSetup {
    CgScal *dev = nullptr;
    std::vector<CgScal> host;
    size_t used = 0;
};

template <typename T> void alloc_cg(Ctx &c, CgWs<T> &w, size_t m, ScalSetup &ss) {
    Arena &a = c.arena;
    w.x = a.alloc<T>(m);
    w.r = a.alloc<T>(m);
    w.z = a.alloc<T>(m);
    w.p0 = a.alloc<T>(m);
    w.p1 = a.alloc<T>(m);
    w.q = a.alloc<T>(m);
    if (ss.used >= ss.host.size()) fail(AMG_ERR_HIP, "CG scalar blocks miscounted");
    w.sc = ss.dev + ss.used;
    w.hmail = take_mail(c, &ss.host[ss.used].mail);
    ++ss.used;
}

template <typename T> void alloc_vc(Arena &a, VcWs<T> &v, size_t m) {
    v.b = a.alloc<T>(m);
    v.x = a.alloc<T>(m);
    v.r = a.alloc<T>(m);
    v.x2 = a.alloc<T>(m);
    v.t = a.alloc<T>(m);
}

void alloc_workspaces(Ctx &c) {
    Arena &a = c.arena;
    AMG_HIP(hipStreamSynchronize(c.stream));
    const int nbp = c.nbp;
    c.ws.assign(c.L, LevelWs{});
    const bool mixed = c.o.inner_precision == 32;
    ScalSetup ss;
    ss.host.assign((size_t)c.L * (mixed ? 6 : 4) + 1, CgScal{});
    ss.dev = a.alloc<CgScal>(ss.host.size());
    for (int l = 0; l < c.L; ++l) {
        LevelWs &w = c.ws[l];
        const size_t m = (size_t)c.lev[l].n * nbp;
        alloc_cg(c, w.in64, m, ss);
        alloc_cg(c, w.mass, m, ss);
        alloc_cg(c, w.hcg, m, ss);
        alloc_cg(c, w.mass2, m, ss);
        alloc_vc(a, w.vc64, m);
        if (mixed) {
            alloc_cg(c, w.inmx, m, ss);
            alloc_cg(c, w.in32, m, ss);
            alloc_vc(a, w.vc32, m);
            w.rr = a.alloc<double>(m);
            w.b32 = a.alloc<float>(m);
            w.d32 = a.alloc<float>(m);
        }
        w.hf = a.alloc<double>(m);
        w.hy = a.alloc<double>(m);
        w.hw = a.alloc<double>(m);
        w.ht = a.alloc<double>(m);
        w.ml_in = a.alloc<double>(m);
        w.ml_out = a.alloc<double>(m);
        w.ml_mup = a.alloc<double>(m);
        w.ml_mself = a.alloc<double>(m);
        w.ml_z1 = a.alloc<double>(m);
        w.ml_t = a.alloc<double>(m);
    }
    const size_t m0 = (size_t)c.N * nbp;
    alloc_cg(c, c.outer, m0, ss);
    AMG_HIP(hipMemcpyAsync(ss.dev, ss.host.data(), ss.used * sizeof(CgScal), hipMemcpyHostToDevice, c.stream));
    c.ox = a.alloc<double>(m0);
    c.ob = a.alloc<double>(m0);
    c.obq = a.alloc<double>(m0);
    c.pk_in = a.alloc<double>(m0);
    c.pk_out = a.alloc<double>(m0);
    c.tsc = a.alloc<CgScal>(1);
    (void)take_mail(c, &c.tsc_mail);
    c.rsd = a.alloc<RefScal>(1);
    RefScal rs{};
    c.rmail = take_mail(c, &rs.mail);
    AMG_HIP(hipMemcpyAsync(c.rsd, &rs, sizeof(RefScal), hipMemcpyHostToDevice, c.stream));
    AMG_HIP(hipStreamSynchronize(c.stream));  // the host sources of the copies end with this call
}

void fill_info(Ctx &c, amg_info *info, int n, double ms, int outer_it, const double *phase_ms = nullptr) {
    if (!info) return;
    for (int k = 0; k < n; ++k) {
        amg_info &f = info[k];
        std::memset(&f, 0, sizeof(f));
        f.true_rel_resid = -1.0;
        f.bytes_moved = c.st.bytes;
        if (phase_ms)
            for (int q = 0; q < 8; ++q) f.ms_phase[q] = phase_ms[q];
        f.outer_iters = outer_it;
        f.inner_solves = (int)c.st.inner_solves;
        f.inner_iters_total = (int)c.st.inner_iters;
        f.inner_iters_max = (int)c.st.inner_max;
        f.mass_iters_total = (int)c.st.mass_iters;
        f.refine_steps = (int)c.st.refine;
        f.levels = c.L;
        f.ell = c.ell;
        f.ms_total = ms;
    }
}

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

int check_vec_call(Ctx *c, int level, int nb) {
    if (!c) return AMG_ERR_ARG;
    if (level < 0 || level >= c->L) {
        c->err = "level out of range";
        return AMG_ERR_ARG;
    }
    if (nb < 1 || nb > c->nbp || nb > 16) {
        c->err = "nb out of range (1..nb_max)";
        return AMG_ERR_ARG;
    }
    return AMG_OK;
}

// ---------------------------------------------------------------------------
// Measurement only (amg_time_kernel): the cost of a grid-wide synchronisation
// inside one persistent launch against a kernel boundary.  A cooperative
// launch of one workgroup per CU runs `rounds` elementwise steps on v, each
// followed by a grid barrier (release fence, arrival counter, generation
// flag, acquire fence); every wait is bounded (a timed-out wait sets *timeout
// and gives up), so the launch always ends.
__global__ __launch_bounds__(kBlock) void coop_rounds_kernel(int rounds, int n, float *v, unsigned *cnt,
                                                             unsigned *gen, int *timeout) {
    unsigned mygen = 0;
    if (threadIdx.x == 0) mygen = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int t = blockIdx.x * kBlock + threadIdx.x;
    for (int r = 0; r < rounds; ++r) {
        for (int i = t; i < n; i += gridDim.x * kBlock) v[i] = v[i] * 0.5f + 1.0f;
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            const unsigned g0 = mygen;
            if (atomicAdd(cnt, 1u) == gridDim.x - 1) {
                __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __threadfence();
                atomicAdd(gen, 1u);
            } else {
                for (long k = 0; __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0; ++k) {
                    if (k > (1L << 22)) {
                        *timeout = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __threadfence();
            mygen = g0 + 1;
        }
        __syncthreads();
    }
}

// the same elementwise step as one launch (its boundary is the synchronisation)
__global__ __launch_bounds__(kBlock) void step_kernel(int n, float *v) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    for (int i = t; i < n; i += gridDim.x * kBlock) v[i] = v[i] * 0.5f + 1.0f;
}


// ---------------------------------------------------------------------------
// Autotuner of the sparse-product geometry: for every CSR product of a
// context (A_j, S_j, S_j^T, M_j and the fused pass over T_j, per value type and
// at the context's batch width) the lanes per row G = 2^lg are timed over the
// candidates lg = 0 .. the largest with G times the column groups <= 64, with HIP
// events on the context's stream, and the fastest is kept (the default rule's
// choice unless another is more than 2 % faster).  Choices live in a
// process-wide table keyed by device, matrix kind, size, stored entries, batch
// width and value type; amg_autotune fills it (and reads / writes it as JSON),
// amg_setup with opts.autotune = 1 applies what it holds.  The level-0 products
// that run on the sliced-ELL copy (one column) have no such parameter.
struct TuneTable {
    std::mutex m;
    std::map<std::string, int> lg;
    std::map<std::string, std::vector<float>> us;  // timings behind each choice (us per launch)
    static TuneTable &get() {
        static TuneTable *t = new TuneTable();
        return *t;
    }
};

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string tune_key(const std::string &dev, const char *kind, const DCsr &A, int nb, int prec) {
    std::ostringstream k;
    k << "dev=" << dev << ";kind=" << kind << ";n=" << A.n << ";nnz=" << A.nnz << ";nb=" << nb << ";prec=" << prec;
    return k.str();
}

// the table as JSON, one entry per line
void tune_save(const char *path) {
    TuneTable &t = TuneTable::get();
    std::lock_guard<std::mutex> g(t.m);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) fail(AMG_ERR_ARG, std::string("cannot write ") + path);
    std::fprintf(f, "{\"amghess_tune\": 1, \"entries\": [\n");
    size_t k = 0;
    for (const auto &e : t.lg) {
        std::fprintf(f, "  {\"key\": \"%s\", \"lg\": %d, \"us\": [", e.first.c_str(), e.second);
        const auto it = t.us.find(e.first);
        if (it != t.us.end())
            for (size_t q = 0; q < it->second.size(); ++q) std::fprintf(f, "%s%.3f", q ? ", " : "", it->second[q]);
        std::fprintf(f, "]}%s\n", ++k < t.lg.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
    if (std::rename(tmp.c_str(), path) != 0) fail(AMG_ERR_ARG, std::string("cannot write ") + path);
}

// entries of a file written by tune_save (a missing file is an empty table)
void tune_load(const char *path) {
    std::ifstream in(path);
    if (!in) return;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string txt = ss.str();
    TuneTable &t = TuneTable::get();
    std::lock_guard<std::mutex> g(t.m);
    size_t pos = 0;
    for (;;) {
        const size_t k0 = txt.find("\"key\": \"", pos);
        if (k0 == std::string::npos) break;
        const size_t k1 = txt.find('"', k0 + 8);
        const size_t l0 = txt.find("\"lg\": ", k1);
        if (k1 == std::string::npos || l0 == std::string::npos) fail(AMG_ERR_ARG, std::string("malformed ") + path);
        const int lg = std::atoi(txt.c_str() + l0 + 6);
        if (lg < 0 || lg > 6) fail(AMG_ERR_ARG, std::string("malformed ") + path);
        t.lg[txt.substr(k0 + 8, k1 - (k0 + 8))] = lg;
        pos = l0;
    }
}

// Enumerates the tunable products of a context at batch width NB: f(kind,
// matrix, level, prec, is_tpro).
template <int NB, class F> void for_tunables(Ctx &c, F &&f) {
    const int precs[2] = {64, 32};
    for (int pi = 0; pi < 2; ++pi) {
        const int prec = precs[pi];
        if (prec == 32 && c.o.inner_precision != 32) continue;
        for (int l = 0; l < c.L; ++l) {
            Level &Lv = c.lev[l];
            const bool sell = NB == 1 && Lv.A.sl_off;  // level 0: A and M run on the sliced-ELL copy
            const bool sell_vals = prec == 64 ? Lv.A.sl_v != nullptr : Lv.A.sl_v32 != nullptr;
            if (!(sell && sell_vals)) f("A", Lv.A, l, prec, false);
            if (l + 1 < c.L) {
                if (Lv.S.rp) f("S", Lv.S, l, prec, false);
                if (Lv.St.rp) f("St", Lv.St, l, prec, false);
                if (Lv.T.rp && (prec == 64 ? (Lv.T.v && Lv.Ts) : (Lv.T.v32 && Lv.Ts32))) f("T", Lv.T, l, prec, true);
            }
            if (prec == 64 && !(sell && Lv.M.sl_v)) f("M", Lv.M, l, prec, false);
        }
    }
}

// applies the table's entries to the context (no timing)
template <int NB> int tune_apply(Ctx &c) {
    const std::string dev = device_arch();
    TuneTable &t = TuneTable::get();
    std::lock_guard<std::mutex> g(t.m);
    int n = 0;
    for_tunables<NB>(c, [&](const char *kind, DCsr &A, int, int prec, bool) {
        const auto it = t.lg.find(tune_key(dev, kind, A, NB, prec));
        if (it == t.lg.end()) return;
        A.tuned_lg[ilog2(NB)][prec == 32 ? 1 : 0] = (int8_t)it->second;
        ++n;
    });
    return n;
}

// times the candidates of every product the table does not hold yet
template <int NB> int tune_time(Ctx &c, int reps) {
    const std::string dev = device_arch();
    Solver<NB> S(c);
    hipEvent_t e0, e1;
    AMG_HIP(hipEventCreate(&e0));
    AMG_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    // defined (zero) inputs in every buffer the timed products touch
    for (int l = 0; l < c.L; ++l) {
        const size_t m = (size_t)c.lev[l].n * NB;
        LevelWs &w = c.ws[l];
        for (double *p : {w.vc64.x, w.vc64.r, w.vc64.t, w.hf, w.hy}) AMG_HIP(hipMemsetAsync(p, 0, m * 8, c.stream));
        if (c.o.inner_precision == 32)
            for (float *p : {w.vc32.x, w.vc32.r, w.vc32.t}) AMG_HIP(hipMemsetAsync(p, 0, m * 4, c.stream));
    }
    int timed = 0;
    for_tunables<NB>(c, [&](const char *kind, DCsr &A, int l, int prec, bool is_t) {
        const std::string key = tune_key(dev, kind, A, NB, prec);
        {
            TuneTable &t = TuneTable::get();
            std::lock_guard<std::mutex> g(t.m);
            if (t.lg.count(key)) return;
        }
        const int pi = prec == 32 ? 1 : 0, nbi = ilog2(NB);
        const int lgmax = is_t ? 6 - ilog2(NB) : max_lg<NB>();
        // the default rule's choice
        int lg_def;
        if (is_t) {
            const double mm = A.n > 0 ? (double)A.nnz / (double)A.n : 1.0;
            int G = 1;
            while (G * NB < 64 && G < mm / kSpmvUnroll) G <<= 1;
            lg_def = ilog2(G);
        } else {
            lg_def = make_geo<NB>(A.nnz, A.n).lg;
        }
        auto launch = [&](auto tT) {
            using T = decltype(tT);
            Level &Lv = c.lev[l];
            VcWs<T> &v = vcws<T>(c.ws[l]);
            if (is_t) {
                S.template tpro<T, 0>(Lv, vcws<T>(c.ws[l + 1]).x, EProCheb<T, NB>{v.t, v.r, dl1inv<T>(Lv), v.x, T(1)},
                                      nullptr);
            } else if (kind[0] == 'M') {
                S.template spmv<double, 0>(A, A.v, GPlain<double, NB>{c.ws[l].hf}, EStore<double, NB>{c.ws[l].hy},
                                           NoFin{}, nullptr);
            } else {
                const T *x = kind[0] == 'S' && kind[1] == 0 ? vcws<T>(c.ws[l + 1]).x : v.x;
                T *y = kind[0] == 'S' && kind[1] == 't' ? vcws<T>(c.ws[l + 1]).r : v.r;
                S.template spmv<T, 0>(A, avals<T>(A), GPlain<T, NB>{x}, EStore<T, NB>{y}, NoFin{}, nullptr);
            }
        };
        auto once = [&]() {
            if (prec == 64) launch(double{});
            else launch(float{});
        };
        std::vector<float> us;
        for (int lg = 0; lg <= lgmax; ++lg) {
            A.tuned_lg[nbi][pi] = (int8_t)lg;
            once();
            once();
            AMG_HIP(hipEventRecord(e0, c.stream));
            for (int r = 0; r < reps; ++r) once();
            AMG_HIP(hipEventRecord(e1, c.stream));
            AMG_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
            us.push_back(1e3f * ms / reps);
        }
        AMG_HIP(hipGetLastError());
        int best = lg_def;
        for (int lg = 0; lg <= lgmax; ++lg)
            if (us[lg] < 0.98f * us[best] && us[lg] < us[lg_def] * 0.98f) best = lg;
        A.tuned_lg[nbi][pi] = (int8_t)best;
        TuneTable &t = TuneTable::get();
        std::lock_guard<std::mutex> g(t.m);
        t.lg[key] = best;
        t.us[key] = us;
        ++timed;
    });
    c.st.reset();
    return timed;
}

// amg_time_kernel 5 and 6: `reps` rounds of an elementwise step over a float
// vector of 2^16 entries, synchronised grid-wide between rounds, in one
// cooperative launch of one workgroup per CU (5) or as `reps` dependent
// launches of the same grid (6).  *ms_avg: ms per round.
int time_sync(Ctx &c, int which, int reps, double *ms_avg, double *bytes) {
    int dev = 0, ncu = 0;
    AMG_HIP(hipGetDevice(&dev));
    AMG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int n = 1 << 16;
    float *v = c.arena.alloc<float>(n);
    unsigned *w = c.arena.alloc<unsigned>(64);
    int *to = reinterpret_cast<int *>(w + 32);
    AMG_HIP(hipMemsetAsync(v, 0, sizeof(float) * n, c.stream));
    AMG_HIP(hipMemsetAsync(w, 0, 64 * sizeof(unsigned), c.stream));
    hipEvent_t e0, e1;
    AMG_HIP(hipEventCreate(&e0));
    AMG_HIP(hipEventCreate(&e1));
    unsigned *cnt = w, *gen = w + 16;
    void *args[] = {(void *)&reps, (void *)&n, (void *)&v, (void *)&cnt, (void *)&gen, (void *)&to};
    auto run = [&]() {
        if (which == 5)
            AMG_HIP(hipLaunchCooperativeKernel((const void *)coop_rounds_kernel, dim3(ncu), dim3(kBlock), args, 0,
                                               c.stream));
        else
            for (int r = 0; r < reps; ++r)
                hipLaunchKernelGGL(step_kernel, dim3(ncu), dim3(kBlock), 0, c.stream, n, v);
        AMG_HIP(hipGetLastError());
    };
    run();  // warm-up
    AMG_HIP(hipEventRecord(e0, c.stream));
    run();
    AMG_HIP(hipEventRecord(e1, c.stream));
    AMG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int h_to = 0;
    AMG_HIP(hipMemcpy(&h_to, to, sizeof(int), hipMemcpyDeviceToHost));
    c.arena.release(v);
    c.arena.release(w);
    if (h_to) fail(AMG_ERR_NOCONV, "a grid barrier wait timed out");
    *ms_avg = ms / reps;
    if (bytes) *bytes = 2.0 * sizeof(float) * n;
    return AMG_OK;
}

}  // namespace
}  // namespace amg

using namespace amg;

struct amg_ctx {
    Ctx c;
};

extern "C" {

int amg_opts_default(amg_opts *o) {
    if (!o) return AMG_ERR_ARG;
    std::memset(o, 0, sizeof(*o));
    o->beta = 1e-2;
    o->hess_levels = 0;
    o->auto_levels = 1;
    o->max_levels = 10;
    o->max_coarse = 200;
    o->dense_max = 4096;
    o->theta0 = 0.08;
    o->agg_seed = 0x200111533ull;
    o->nu = 1;
    o->inner_rtol = 1e-8;
    o->mass_rtol = 1e-8;
    o->precond_inner_rtol = 1e-8;
    o->inner_maxit = 500;
    o->mass_maxit = 500;
    o->outer_maxit = 200;
    o->inner_precision = 64;
    o->inner32_rtol = 1e-6;
    o->refine_maxit = 6;
    o->nb_max = 1;
    o->precond = 1;
    o->check_every = 1;
    o->use_graphs = 2;
    o->coarse_hess_rtol = 1e-4;
    o->dense_solve_max = 2048;
    o->mixed_mode = 0;
    o->smoother = 0;
    o->true_resid = 0;
    o->autotune = 0;
    return AMG_OK;
}

const char *amg_last_error(amg_ctx *ctx) { return ctx ? ctx->c.err.c_str() : g_setup_err.c_str(); }

int amg_setup(const amg_csr *A, const amg_csr *M, const uint8_t *dirichlet, const amg_opts *opts, void *stream,
              amg_ctx **out) {
    if (!out) return AMG_ERR_ARG;
    *out = nullptr;
    g_setup_err.clear();
    if (!A || !M || !A->rowptr || !A->col || !A->val || !M->rowptr || !M->col || !M->val) {
        g_setup_err = "null matrix argument";
        return AMG_ERR_ARG;
    }
    if (A->nrows <= 0 || A->nrows != A->ncols || M->nrows != A->nrows || M->ncols != A->ncols || A->nnz <= 0 ||
        M->nnz <= 0) {
        g_setup_err = "matrix sizes invalid or mismatching";
        return AMG_ERR_ARG;
    }
    amg_opts o;
    if (opts) o = *opts;
    else amg_opts_default(&o);
    if (!(o.beta > 0.0) || o.nb_max < 1 || o.nb_max > 16 || o.max_levels < 1 || o.max_coarse < 1 ||
        o.dense_max < 1 || o.dense_max > 4096 || (o.inner_precision != 32 && o.inner_precision != 64) ||
        o.nu != 1 || o.inner_maxit < 1 || o.mass_maxit < 1 || o.outer_maxit < 1 || o.hess_levels < 0 ||
        !(o.theta0 >= 0.0) || o.refine_maxit < 1 || o.use_graphs < 0 || o.use_graphs > 2 ||
        !(o.coarse_hess_rtol > 0.0) || o.dense_solve_max < 0 || o.dense_solve_max > 4096 || o.mixed_mode < 0 ||
        o.mixed_mode > 1 || o.smoother < 0 || o.smoother > 1 || o.true_resid < 0 || o.true_resid > 1 ||
        o.autotune < 0 || o.autotune > 1) {
        g_setup_err = "invalid options (beta > 0, 1 <= nb_max <= 16, dense_max <= 4096, nu = 1, precision 32/64)";
        return AMG_ERR_ARG;
    }
    amg_ctx *h = new (std::nothrow) amg_ctx;
    if (!h) return AMG_ERR_OOM;
    Ctx &c = h->c;
    c.o = o;
    c.stream = reinterpret_cast<hipStream_t>(stream);
    c.nbp = pad_nb(o.nb_max);
    Range rg("amg_setup");
    int rc = guarded(nullptr, [&]() {
        c.lev.reserve(o.max_levels + 1);
        for (auto &p : c.part) p = c.arena.alloc<double>((size_t)2 * 16 * kMaxGrid);
        for (auto &p : c.part2) p = c.arena.alloc<double>((size_t)2 * 16 * kMaxGrid);
        c.dscratch = c.arena.alloc<double>(64);
        c.iscratch = c.arena.alloc<int>(64);
        c.iscratch2 = c.arena.alloc<int>(64);
        AMG_HIP(hipHostMalloc((void **)&c.hsc, sizeof(CgScal), hipHostMallocDefault));
        AMG_HIP(hipHostMalloc((void **)&c.hscr, 64 * sizeof(double), hipHostMallocDefault));
        AMG_HIP(hipHostMalloc((void **)&c.hiscr, 64 * sizeof(int), hipHostMallocDefault));
        AMG_HIP(hipHostMalloc((void **)&c.hiscr2, 64 * sizeof(int), hipHostMallocDefault));
        AMG_HIP(hipHostMalloc((void **)&c.mails, 64 * sizeof(Mail), hipHostMallocDefault));
        AMG_HIP(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
        AMG_HIP(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
        AMG_HIP(hipStreamCreateWithFlags(&c.gal, hipStreamNonBlocking));
        for (auto &e : c.gal_ev) AMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (auto &e : c.poll_ev) AMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (auto &e : c.side_ev) AMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (auto &e : c.poll_ev2) AMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (auto &e : c.mass_ev) AMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        build_hierarchy(c, *A, *M, dirichlet);
        form_dense_hessian(c, o.hess_levels > 0 ? o.hess_levels : c.L);
        alloc_workspaces(c);
        if (o.autotune) dispatch_nb(c.nbp, [&](auto tag) { return tune_apply<decltype(tag)::value>(c); });
        AMG_HIP(hipStreamSynchronize(c.stream));
        return AMG_OK;
    });
    if (rc != AMG_OK) {
        amg_destroy(h);
        return rc;
    }
    *out = h;
    return AMG_OK;
}

int amg_destroy(amg_ctx *ctx) {
    if (!ctx) return AMG_OK;
    Ctx &c = ctx->c;
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    if (c.side) (void)hipStreamSynchronize(c.side);  // setup that failed before joining it
    if (c.gal) (void)hipStreamSynchronize(c.gal);
    c.arena.free_all();
    if (c.hsc) (void)hipHostFree(c.hsc);
    if (c.hscr) (void)hipHostFree(c.hscr);
    if (c.hiscr) (void)hipHostFree(c.hiscr);
    if (c.hiscr2) (void)hipHostFree(c.hiscr2);
    if (c.mails) (void)hipHostFree(c.mails);
    for (auto g : c.graphs) (void)hipGraphExecDestroy(g);
    for (auto e : c.poll_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto e : c.side_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto e : c.poll_ev2)
        if (e) (void)hipEventDestroy(e);
    for (auto e : c.mass_ev)
        if (e) (void)hipEventDestroy(e);
    c.ph.destroy();
    if (c.cap_stream) (void)hipStreamDestroy(c.cap_stream);
    if (c.side) (void)hipStreamDestroy(c.side);
    if (c.gal) (void)hipStreamDestroy(c.gal);
    for (auto e : c.gal_ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
    return AMG_OK;
}

int amg_release_memory(void) {
    DevPool::get().release(-1);
    return AMG_OK;
}

int state_solve(amg_ctx *ctx, int level, const double *u, double *y, int nb, amg_info *info) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, level, nb)) return e;
    if (!u || !y) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        auto t0 = clk::now();
        c.st.reset();
        const int n = c.lev[level].n;
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            S.template elem<0>(n, OpPack<NB>{c.pk_in, u, nb}, NoFin{}, nullptr);
            S.state_solve(level, c.pk_in, c.pk_out, c.o.inner_rtol);
            S.template elem<0>(n, OpUnpack<NB>{y, c.pk_out, nb}, NoFin{}, nullptr);
            AMG_HIP(hipStreamSynchronize(c.stream));
            fill_info(c, info, 1, ms_since(t0), 0);
            return AMG_OK;
        });
    });
}

int adjoint_solve(amg_ctx *ctx, int level, const double *w, double *z, int nb, amg_info *info) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, level, nb)) return e;
    if (!w || !z) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        auto t0 = clk::now();
        c.st.reset();
        const int n = c.lev[level].n;
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            S.template elem<0>(n, OpPack<NB>{c.pk_in, w, nb}, NoFin{}, nullptr);
            S.adjoint_solve(level, c.pk_in, c.pk_out, c.o.inner_rtol);
            S.template elem<0>(n, OpUnpack<NB>{z, c.pk_out, nb}, NoFin{}, nullptr);
            AMG_HIP(hipStreamSynchronize(c.stream));
            fill_info(c, info, 1, ms_since(t0), 0);
            return AMG_OK;
        });
    });
}

int hessian_apply(amg_ctx *ctx, int level, const double *u, double *Hu, int nb, amg_info *info) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, level, nb)) return e;
    if (!u || !Hu) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        auto t0 = clk::now();
        c.st.reset();
        const int n = c.lev[level].n;
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            S.template elem<0>(n, OpPack<NB>{c.pk_in, u, nb}, NoFin{}, nullptr);
            S.hessian_apply(level, c.pk_in, c.pk_out, c.o.inner_rtol, nullptr);
            S.template elem<0>(n, OpUnpack<NB>{Hu, c.pk_out, nb}, NoFin{}, nullptr);
            AMG_HIP(hipStreamSynchronize(c.stream));
            fill_info(c, info, 1, ms_since(t0), 0);
            return AMG_OK;
        });
    });
}

int hessian_precond_apply(amg_ctx *ctx, const double *r, double *z, int nb, amg_info *info) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, 0, nb)) return e;
    if (!r || !z) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        auto t0 = clk::now();
        c.st.reset();
        const int n = c.N;
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            S.template elem<0>(n, OpPack<NB>{c.pk_in, r, nb}, NoFin{}, nullptr);
            S.Bop(0, c.pk_in, c.pk_out);
            S.template elem<0>(n, OpUnpack<NB>{z, c.pk_out, nb}, NoFin{}, nullptr);
            AMG_HIP(hipStreamSynchronize(c.stream));
            fill_info(c, info, 1, ms_since(t0), 0);
            return AMG_OK;
        });
    });
}

int reduced_solve(amg_ctx *ctx, const double *yd, const double *u0, double *u, int nb, double rtol,
                  amg_info *info) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, 0, nb)) return e;
    if (!yd || !u || !(rtol > 0.0)) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    Range rg("reduced_solve");
    return guarded(&c, [&]() {
        auto t0 = clk::now();
        c.st.reset();
        if (info) c.ph.start();
        struct PhOff {  // no phase marks after an error either
            PhaseTimer &p;
            ~PhOff() { p.on = false; }
        } ph_off{c.ph};
        const int n = c.N;
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            // b = K^T M_y y_d
            c.ph.mark(kPhRhs, c.stream);
            {
                Range rr("rhs");
                S.template elem<0>(n, OpPack<NB>{c.pk_in, yd, nb}, NoFin{}, nullptr);
                S.mass_apply(0, 1, c.pk_in, c.obq, nullptr, nullptr);
                S.adjoint_solve(0, c.obq, c.ob, c.o.inner_rtol);
            }
            c.ph.mark(kPhOuter, c.stream);
            if (u0) S.template elem<0>(n, OpPack<NB>{c.ox, u0, nb}, NoFin{}, nullptr);
            int it = 0;
            const int rc = S.outer(c.ob, c.ox, u0 != nullptr, rtol, nb, &it);
            // the true residual b - H u at exit (one more Hessian action)
            const bool true_res = info && c.o.true_resid && (rc == AMG_OK || rc == AMG_ERR_NOCONV);
            if (true_res) {
                c.ph.mark(kPhTrue, c.stream);
                Range rt("true_residual");
                S.hessian_apply(0, c.ox, c.pk_out, c.o.inner_rtol, c.ob);
                S.template elem<2>(n, OpDot<NB>{c.pk_out, c.pk_out, c.ob, c.ob}, FinStore<NB>{c.dscratch}, nullptr);
                AMG_HIP(hipMemcpyAsync(c.hscr, c.dscratch, 2 * NB * sizeof(double), hipMemcpyDeviceToHost,
                                       c.stream));
            }
            c.ph.mark(kPhEnd, c.stream);
            S.template elem<0>(n, OpUnpack<NB>{u, c.ox, nb}, NoFin{}, nullptr);
            AMG_HIP(hipStreamSynchronize(c.stream));
            double pms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (info) c.ph.sum(pms);
            fill_info(c, info, nb, ms_since(t0), it, pms);
            if (info) {
                if (true_res)
                    for (int k = 0; k < nb; ++k)
                        info[k].true_rel_resid =
                            c.hscr[NB + k] > 0 ? std::sqrt(c.hscr[k] / c.hscr[NB + k]) : 0.0;
                S.read_sc(c.outer.sc);
                for (int k = 0; k < nb; ++k) {
                    const ColScal &cs = c.hsc->s[k];
                    info[k].rel_resid = cs.bb > 0 ? std::sqrt(cs.rr / cs.bb) : 0.0;
                    info[k].status_detail = cs.iters;
                }
            }
            if (rc == AMG_ERR_NOCONV) c.err = "outer CG reached outer_maxit";
            if (rc == AMG_ERR_INDEFINITE) c.err = "indefinite preconditioner";
            return rc;
        });
    });
}

int reduced_objective(amg_ctx *ctx, const double *u, const double *yd, double *J_host, double *grad, int nb,
                      amg_info *info) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, 0, nb)) return e;
    if (!u || !yd || (!J_host && !grad)) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        auto t0 = clk::now();
        c.st.reset();
        const int n = c.N;
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            LevelWs &w = c.ws[0];
            S.template elem<0>(n, OpPack<NB>{c.pk_in, u, nb}, NoFin{}, nullptr);
            S.template elem<0>(n, OpPack<NB>{c.obq, yd, nb}, NoFin{}, nullptr);
            S.state_solve(0, c.pk_in, c.ox, c.o.inner_rtol);                                        // y = K u
            S.template elem<0>(n, OpAxpby<NB>{c.ox, c.ox, c.obq, 1.0, -1.0}, NoFin{}, nullptr);     // e = y - y_d
            S.mass_apply(0, 1, c.ox, c.ob, c.ox, c.dscratch);                                       // M_y e, e.M_y e
            S.mass_apply(0, 0, c.pk_in, c.pk_out, c.pk_in, c.dscratch + 16);                        // u.M_u u
            if (J_host) {
                AMG_HIP(hipMemcpyAsync(c.hscr, c.dscratch, 32 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
                AMG_HIP(hipStreamSynchronize(c.stream));
                for (int k = 0; k < nb; ++k) J_host[k] = 0.5 * c.hscr[k] + 0.5 * c.o.beta * c.hscr[16 + k];
            }
            if (grad) {
                // grad = M (D A^{-1} M_y e) + beta M u
                S.solve_A(0, c.ob, w.ht, c.o.inner_rtol);
                const uint8_t *mk = c.has_mask ? c.mask0 : nullptr;
                S.template spmv<double, 0>(c.lev[0].M, c.lev[0].M.v, GLin<NB>{w.ht, mk, c.pk_in, c.o.beta},
                                           ELin<NB>{c.pk_out, nullptr, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr},
                                           NoFin{}, nullptr);
                S.template elem<0>(n, OpUnpack<NB>{grad, c.pk_out, nb}, NoFin{}, nullptr);
            }
            AMG_HIP(hipStreamSynchronize(c.stream));
            fill_info(c, info, 1, ms_since(t0), 0);
            return AMG_OK;
        });
    });
}

int amg_mass_apply(amg_ctx *ctx, int level, int which, const double *x, double *y, int nb) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, level, nb)) return e;
    if (!x || !y || which < 0 || which > 3) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        const int n = c.lev[level].n;
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            S.template elem<0>(n, OpPack<NB>{c.pk_in, x, nb}, NoFin{}, nullptr);
            S.mass_apply(level, which, c.pk_in, c.pk_out, nullptr, nullptr);
            S.template elem<0>(n, OpUnpack<NB>{y, c.pk_out, nb}, NoFin{}, nullptr);
            AMG_HIP(hipStreamSynchronize(c.stream));
            return AMG_OK;
        });
    });
}

int amg_mass_quad(amg_ctx *ctx, int which, const double *x, double *q_host, int nb) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, 0, nb)) return e;
    if (!x || !q_host || which < 0 || which > 1) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        const int n = c.N;
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            S.template elem<0>(n, OpPack<NB>{c.pk_in, x, nb}, NoFin{}, nullptr);
            S.mass_apply(0, which, c.pk_in, c.pk_out, c.pk_in, c.dscratch);
            AMG_HIP(hipMemcpyAsync(c.hscr, c.dscratch, 16 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
            AMG_HIP(hipStreamSynchronize(c.stream));
            for (int k = 0; k < nb; ++k) q_host[k] = c.hscr[k];
            return AMG_OK;
        });
    });
}

int amg_num_levels(amg_ctx *ctx, int32_t *L, int32_t *ell) {
    if (!ctx) return AMG_ERR_ARG;
    if (L) *L = ctx->c.L;
    if (ell) *ell = ctx->c.ell;
    return AMG_OK;
}

int amg_level_size(amg_ctx *ctx, int level, int32_t *n, int32_t *nnzA, int32_t *nnzS, int32_t *nnzM) {
    if (!ctx || level < 0 || level >= ctx->c.L) return AMG_ERR_ARG;
    const Level &L = ctx->c.lev[level];
    if (n) *n = L.n;
    if (nnzA) *nnzA = L.A.nnz;
    if (nnzS) *nnzS = L.S.nnz;
    if (nnzM) *nnzM = L.M.nnz;
    return AMG_OK;
}

int amg_copy_aggregates(amg_ctx *ctx, int level, int32_t *agg, uint8_t *root) {
    if (!ctx || level < 0 || level >= ctx->c.L - 1) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        const Level &L = c.lev[level];
        if (agg) AMG_HIP(hipMemcpy(agg, L.agg, sizeof(int) * L.n, hipMemcpyDeviceToHost));
        if (root) AMG_HIP(hipMemcpy(root, L.root, L.n, hipMemcpyDeviceToHost));
        return AMG_OK;
    });
}

int amg_copy_csr(amg_ctx *ctx, int level, int which, int32_t *rowptr, int32_t *col, double *val) {
    if (!ctx || level < 0 || level >= ctx->c.L || which < 0 || which > 3) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    const Level &L = c.lev[level];
    const DCsr &m = which == 0 ? L.A : which == 1 ? L.S : which == 2 ? L.St : L.M;
    if (!m.rp) return AMG_ERR_ARG;
    return guarded(&c, [&]() {
        AMG_HIP(hipStreamSynchronize(c.stream));
        if (rowptr) AMG_HIP(hipMemcpy(rowptr, m.rp, sizeof(int) * (m.n + 1), hipMemcpyDeviceToHost));
        if (col) AMG_HIP(hipMemcpy(col, m.ci, sizeof(int) * m.nnz, hipMemcpyDeviceToHost));
        if (val) AMG_HIP(hipMemcpy(val, m.v, sizeof(double) * m.nnz, hipMemcpyDeviceToHost));
        return AMG_OK;
    });
}

int amg_copy_dense(amg_ctx *ctx, int which, int32_t *n, double *out) {
    if (!ctx || which < 0 || which > 2) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    const int m = which == 0 ? c.nAinv : c.nH;
    if (n) *n = m;
    if (!out) return AMG_OK;
    const double *src = which == 0 ? c.Ainv : which == 1 ? c.Hdense : c.Hinv;
    return guarded(&c, [&]() {
        AMG_HIP(hipStreamSynchronize(c.stream));
        AMG_HIP(hipMemcpy(out, src, sizeof(double) * m * m, hipMemcpyDeviceToHost));
        return AMG_OK;
    });
}

int amg_set_hess_levels(amg_ctx *ctx, int ell) {
    if (!ctx || ell < 1 || ell > ctx->c.L) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        form_dense_hessian(c, ell);
        return AMG_OK;
    });
}

int amg_hierarchy_quality(amg_ctx *ctx, int level, const double *v0, int iters, double *a_tilde) {
    if (!ctx || !v0 || !a_tilde || iters < 1 || level < 0 || level + 1 >= ctx->c.L) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        c.st.reset();
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            const int j = level, n = c.lev[j].n;
            Level &L = c.lev[j];
            LevelWs &w0 = c.ws[j], &w1 = c.ws[j + 1];
            const double rtol = c.o.inner_rtol;
            double *v = w0.ml_in, *y = w0.ml_z1, *d = c.dscratch;
            auto restrict_ = [&](const double *x, double *out) {
                S.template spmv<double, 0>(L.St, L.St.v, GPlain<double, NB>{x}, EStore<double, NB>{out}, NoFin{},
                                           nullptr);
            };
            auto prolong = [&](const double *x, double *out) {
                S.template spmv<double, 0>(L.S, L.S.v, GPlain<double, NB>{x}, EStore<double, NB>{out}, NoFin{},
                                           nullptr);
            };
            auto dots = [&](const double *a, const double *b, const double *p, const double *q) {
                S.template elem<2>(n, OpDot<NB>{a, b, p, q}, FinStore<NB>{d}, nullptr);
                AMG_HIP(hipMemcpyAsync(c.hscr, d, 2 * NB * sizeof(double), hipMemcpyDeviceToHost, c.stream));
                AMG_HIP(hipStreamSynchronize(c.stream));
            };
            // v = v0 / ||v0|| in column 0 (the other columns stay zero)
            S.template elem<0>(n, OpPack<NB>{v, v0, 1}, NoFin{}, nullptr);
            dots(v, v, v, v);
            if (!(c.hscr[0] > 0.0)) fail(AMG_ERR_ARG, "v0 is zero");
            S.template elem<0>(n, OpAxpby<NB>{v, v, nullptr, 1.0 / std::sqrt(c.hscr[0]), 0.0}, NoFin{}, nullptr);
            double lam = 0.0;
            for (int it = 0; it < iters; ++it) {
                // E v = K_j v - S_j K_{j+1} M_{j+1}^{-1} S_j^T M_j v
                S.mass_apply(j, 0, v, w0.ml_out, nullptr, nullptr);
                restrict_(w0.ml_out, w1.ml_in);
                S.mass_solve(j + 1, w1.ml_in, w1.ml_mup);
                S.state_solve(j + 1, w1.ml_mup, w1.ml_out, rtol);
                prolong(w1.ml_out, w0.ml_mup);
                S.state_solve(j, v, w0.ml_mself, rtol);
                S.template elem<0>(n, OpAxpby<NB>{w0.ml_t, w0.ml_mself, w0.ml_mup, 1.0, -1.0}, NoFin{}, nullptr);
                // y = E^T (E v) = K_j^T e - M_j S_j M_{j+1}^{-1} K_{j+1}^T S_j^T e
                restrict_(w0.ml_t, w1.ml_in);
                S.adjoint_solve(j + 1, w1.ml_in, w1.ml_out, rtol);
                S.mass_solve(j + 1, w1.ml_out, w1.ml_mup);
                prolong(w1.ml_mup, w0.ml_mup);
                S.mass_apply(j, 0, w0.ml_mup, w0.ml_out, nullptr, nullptr);
                S.adjoint_solve(j, w0.ml_t, w0.ml_mself, rtol);
                S.template elem<0>(n, OpAxpby<NB>{y, w0.ml_mself, w0.ml_out, 1.0, -1.0}, NoFin{}, nullptr);
                // Rayleigh quotient and the next iterate
                dots(v, y, y, y);
                lam = c.hscr[0];
                const double ny = std::sqrt(c.hscr[NB]);
                if (!(ny > 0.0)) break;
                S.template elem<0>(n, OpAxpby<NB>{v, y, nullptr, 1.0 / ny, 0.0}, NoFin{}, nullptr);
            }
            *a_tilde = std::sqrt(std::max(lam, 0.0));
            return AMG_OK;
        });
    });
}

int amg_autotune(amg_ctx *ctx, int reps, const char *cache_path, int32_t *n_timed) {
    if (!ctx || reps < 1) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    return guarded(&c, [&]() {
        if (cache_path) tune_load(cache_path);
        int timed = 0;
        dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            timed = tune_time<NB>(c, reps);
            tune_apply<NB>(c);
            return AMG_OK;
        });
        if (cache_path) tune_save(cache_path);
        if (n_timed) *n_timed = timed;
        return AMG_OK;
    });
}

int amg_vcycle_apply(amg_ctx *ctx, int level, int prec, const double *b, double *x, int nb) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, level, nb)) return e;
    if (!b || !x || (prec != 32 && prec != 64)) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    if (prec == 32 && c.o.inner_precision != 32) {
        c.err = "the float32 V-cycle needs inner_precision = 32";
        return AMG_ERR_ARG;
    }
    return guarded(&c, [&]() {
        const int n = c.lev[level].n;
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            auto run = [&](auto tT) {
                using T = decltype(tT);
                VcWs<T> &v = vcws<T>(c.ws[level]);
                // the first smoothing iterate is needed only where the cycle smooths
                const bool smooths = level < c.L - 1 && !c.lev[level].Ainv;
                S.template elem<0>(n, OpVcIn<T, NB>{v.b, smooths ? v.x : nullptr, b, dl1inv<T>(c.lev[level]),
                                                    (T)S.first_scale(), nb},
                                   NoFin{}, nullptr);
                if (smooths) S.template vcycle<T>(level, v.b, v.x2, false, nullptr);
                else S.template dense_apply<T>(level == c.L - 1 ? c.dAc : c.lev[level].dA, v.b, v.x2, nullptr);
                S.template elem<0>(n, OpVcOut<T, NB>{x, v.x2, nb}, NoFin{}, nullptr);
            };
            if (prec == 64) run(double{});
            else run(float{});
            AMG_HIP(hipStreamSynchronize(c.stream));
            return AMG_OK;
        });
    });
}

int amg_time_kernel(amg_ctx *ctx, int which, int prec, int nb, int reps, double *ms_avg, double *bytes) {
    if (int e = check_vec_call(ctx ? &ctx->c : nullptr, 0, nb)) return e;
    if (which < 0 || which > 6 || (prec != 32 && prec != 64) || reps < 1 || !ms_avg) return AMG_ERR_ARG;
    Ctx &c = ctx->c;
    if (prec == 32 && c.o.inner_precision != 32) {
        c.err = "float32 kernels need inner_precision = 32";
        return AMG_ERR_ARG;
    }
    if (c.L < 2 && (which == 1 || which == 2 || which == 3)) return AMG_ERR_ARG;
    if (which == 4 && (prec != 64 || c.o.inner_precision != 32 || c.o.mixed_mode != 0)) {
        c.err = "the CG product of the float32-preconditioned FP64 CG needs prec 64, inner_precision 32, mixed_mode 0";
        return AMG_ERR_ARG;
    }
    if (which >= 5) return guarded(&c, [&]() { return time_sync(c, which, reps, ms_avg, bytes); });
    if (which == 3) {
        const Level &L0 = c.lev[0];
        const bool has = L0.T.rp && (prec == 64 ? (L0.T.v && L0.Ts) : (L0.T.v32 && L0.Ts32));
        if (!has) {
            c.err = "level 0 keeps no T = A S for the fused coarse correction";
            return AMG_ERR_ARG;
        }
    }
    return guarded(&c, [&]() {
        return dispatch_nb(c.nbp, [&](auto tag) {
            constexpr int NB = decltype(tag)::value;
            Solver<NB> S(c);
            const Level &L0 = c.lev[0];
            const int n = L0.n;
            const double sz = prec == 64 ? 8.0 : 4.0;
            const double nbd = NB;
            // algorithmic bytes: row pointers, (col, val) per stored entry, x read
            // once, y written once (per column); a column takes 2 bytes in the
            // level-0 sliced-ELL copy (single column), else 4
            auto ib = [&](int l) { return l == 0 && NB == 1 && c.lev[0].A.sl_off ? 2.0 : 4.0; };
            const double spmv_b = 4.0 * (n + 1) + (ib(0) + sz) * L0.A.nnz + 2.0 * sz * n * nbd;
            hipEvent_t e0, e1;
            AMG_HIP(hipEventCreate(&e0));
            AMG_HIP(hipEventCreate(&e1));
            // single kernels (which 0, 1): launch r serves its slices from XCD
            // ranges rotated by r mod 8, so that no launch finds its share of
            // the level-0 matrix in the L2 of the XCD the launch before left it
            // in (back to back it would, unlike the launches in a solve, which
            // other work separates)
            const bool rotate = which < 2 || which == 4;
            // entry 4 folds the finalize into the product exactly when a solve does
            // (when every workgroup can afford to sum the partials it needs)
            bool fused4 = false;
            {
                long q = (long)grid_rows((long)n * NB, kBlock, red_grid_max<NB>()) * NB;
                q += (long)S.template red_grid<float>(L0.A) * NB;
                fused4 = q <= kFusedPartials;
            }
            auto run = [&](auto tT) {
                using T = decltype(tT);
                VcWs<T> &v = vcws<T>(c.ws[0]);
                auto once = [&]() {
                    if (which == 0)
                        S.template spmv<T, 0>(L0.A, avals<T>(L0.A), GPlain<T, NB>{v.x}, EStore<T, NB>{v.r}, NoFin{},
                                              nullptr);
                    else if (which == 1)  // the pre-sweep residual r = b - A x, x = D^{-1} b given
                        S.template spmv<T, 0>(L0.A, avals<T>(L0.A), GPlain<T, NB>{v.x}, EResB<T, NB>{v.b, v.r},
                                              NoFin{}, nullptr);
                    else if (which == 3)  // coarse correction t += S e fused with the first post step
                        S.template tpro<T, 0>(L0, vcws<T>(c.ws[1]).x,
                                              EProCheb<T, NB>{v.t, v.r, dl1inv<T>(L0), v.x, T(1)}, nullptr);
                    else if (which == 4) {  // the inner CG's product q = A z + beta q_old with its
                                            // folded finalize, as in every iteration of a solve
                        if constexpr (std::is_same_v<T, double>) {
                            CgWs<double> &w = c.ws[0].inmx;
                            const GZ<double, NB, float> gz{c.ws[0].d32};
                            const ECgQR<double, NB, float> ep{c.ws[0].d32, w.p0, w.p1, w.q, c.tsc};
                            if (fused4) {
                                const FusedFin<NB, false> pro{c.tsc, c.part[1], c.pgrid[1], c.part[2], c.pgrid[2]};
                                S.template spmv<double, 1>(L0.A, L0.A.v, gz, ep, NoFin{}, &c.tsc->all_conv, 0, pro);
                            } else {
                                S.template spmv<double, 1>(L0.A, L0.A.v, gz, ep, NoFin{}, &c.tsc->all_conv, 0);
                            }
                        }
                    }
                    else
                        S.template vcycle<T>(0, v.b, v.x2, false, nullptr);
                };
                // defined inputs
                AMG_HIP(hipMemsetAsync(v.x, 0, sizeof(T) * n * NB, c.stream));
                AMG_HIP(hipMemsetAsync(v.b, 0, sizeof(T) * n * NB, c.stream));
                if (which == 4) {
                    // a CG that never converges: the folded finalize sums partials of
                    // ones (r.r > 0 = tolerance, r.z > 0) over as many workgroups as in
                    // a solve, and beta = r.z / rho = 1; z, p and q start at zero
                    CgWs<double> &w = c.ws[0].inmx;
                    AMG_HIP(hipMemsetAsync(c.ws[0].d32, 0, sizeof(float) * n * NB, c.stream));
                    AMG_HIP(hipMemsetAsync(w.p0, 0, sizeof(double) * n * NB, c.stream));
                    AMG_HIP(hipMemsetAsync(w.q, 0, sizeof(double) * n * NB, c.stream));
                    const int g = grid_rows((long)n * NB, kBlock, red_grid_max<NB>());
                    S.pgrid[1] = g;
                    S.pgrid[2] = S.template red_grid<float>(L0.A);
                    std::vector<double> ones((size_t)2 * 16 * kMaxGrid, 1.0);
                    AMG_HIP(hipMemcpyAsync(c.part[1], ones.data(), ones.size() * sizeof(double),
                                           hipMemcpyHostToDevice, c.stream));
                    AMG_HIP(hipMemcpyAsync(c.part[2], ones.data(), ones.size() * sizeof(double),
                                           hipMemcpyHostToDevice, c.stream));
                    CgScal h{};
                    for (int col = 0; col < 16; ++col) {
                        ColScal &cs = h.s[col];
                        cs.conv = col < NB ? 0 : 1;
                        cs.tol2 = 0.0;
                        cs.rho = (double)S.pgrid[2];
                        cs.rho_next = cs.rho;
                        cs.beta = 1.0;
                    }
                    h.nb = NB;
                    h.mail = c.tsc_mail;
                    AMG_HIP(hipMemcpyAsync(c.tsc, &h, sizeof(CgScal), hipMemcpyHostToDevice, c.stream));
                    AMG_HIP(hipStreamSynchronize(c.stream));
                }
                if (which == 3) {
                    AMG_HIP(hipMemsetAsync(v.t, 0, sizeof(T) * n * NB, c.stream));
                    AMG_HIP(hipMemsetAsync(v.r, 0, sizeof(T) * n * NB, c.stream));
                    AMG_HIP(hipMemsetAsync(vcws<T>(c.ws[1]).x, 0, sizeof(T) * c.lev[1].n * NB, c.stream));
                }
                once();
                AMG_HIP(hipStreamSynchronize(c.stream));
                AMG_HIP(hipEventRecord(e0, c.stream));
                for (int r = 0; r < reps; ++r) {
                    if (rotate) S.xrot = (r + 1) % kXcd;
                    once();
                }
                S.xrot = 0;
                AMG_HIP(hipEventRecord(e1, c.stream));
                AMG_HIP(hipEventSynchronize(e1));
            };
            if (prec == 64) run(double{});
            else run(float{});
            float ms = 0.f;
            AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            *ms_avg = ms / reps;
            if (bytes) {
                if (which == 0) *bytes = spmv_b;
                else if (which == 4)  // the method's q = A p in FP64 (int32 columns counted)
                    *bytes = spmv_bytes(n, L0.A.nnz, 8, NB);
                else if (which == 1)  // gathers x once, reads b, writes r
                    *bytes = 4.0 * (n + 1) + (ib(0) + sz) * L0.A.nnz + 3.0 * sz * n * nbd;
                else if (which == 3)  // T's pattern with both value arrays, e gathered once,
                                      // t, r and dinv read, t and y written
                    *bytes = 4.0 * (n + 1) + ((L0.Tc16 ? 2.0 : 4.0) + 2.0 * sz) * L0.T.nnz +
                             sz * c.lev[1].n * nbd + (4.0 * sz * nbd + sz) * n;
                else {
                    // the cycle ends at the first level with a dense inverse
                    int Lc = c.L - 1;
                    for (int l = 1; l < c.L - 1; ++l)
                        if (c.lev[l].Ainv) {
                            Lc = l;
                            break;
                        }
                    double tot = 0.0;
                    for (int l = 0; l < Lc; ++l) {
                        const Level &Lv = c.lev[l];
                        const double nl = Lv.n, nc = c.lev[l + 1].n;
                        const double a = 4.0 * (nl + 1) + (ib(l) + sz) * Lv.A.nnz;
                        if (c.o.smoother == 1) {
                            // Chebyshev: pre step (x, b, dinv in; t out), residual (t, b in; r
                            // out), post steps (t, b, dinv in; x out) and (x, t, b, dinv in; out)
                            tot += a + sz * nl * nbd * 3 + sz * nl;
                            tot += a + sz * nl * nbd * 3;
                            tot += a + sz * nl * nbd * 3 + sz * nl;
                            tot += a + sz * nl * nbd * 4 + sz * nl;
                        } else {
                            // pre-sweep residual (x gathered, b in, r out), post (x, b, dinv in; out)
                            tot += a + sz * nl * nbd * 3;
                            tot += a + sz * nl * nbd * 3 + sz * nl;
                        }
                        // restriction (with the next level's first iterate when it is
                        // smoothed) and prolongation (+ add)
                        tot += 4.0 * (nc + 1) + (4.0 + sz) * Lv.St.nnz + sz * (nl + nc) * nbd;
                        if (l + 1 < Lc) tot += sz * nc + sz * nc * nbd;
                        tot += 4.0 * (nl + 1) + (4.0 + sz) * Lv.S.nnz + sz * (nc + 2 * nl) * nbd;
                    }
                    const double nc = c.lev[Lc].n;
                    tot += 8.0 * nc * nc + 2.0 * sz * nc * nbd;
                    *bytes = tot;
                }
            }
            return AMG_OK;
        });
    });
}

}  // extern "C"
