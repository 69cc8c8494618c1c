"""Benchmark of the reduced-Hessian solve on one MI355X.

Workload: the 3D unit cube, 64^3 grid split into 6 Kuhn tetrahedra per cube
(274,625 nodes, 1,572,864 P1 elements), log-normal kappa (16 seeded Fourier
modes, variance 1), beta = 1e-3, the manufactured desired state of the paper's
eq. test-state; inner A-solves by FP64 CG preconditioned with float32
V-cycles (the bulk of the traffic; degree-2 Chebyshev smoothing on the l1
diagonal), outer Hessian CG, CG residuals, dot products and dense coarse
factors in FP64; sparse-product geometry from the autotuner.

One step = the whole hot path on that input, resident in HBM when the timed
region starts: the smoothed-aggregation setup on the GPU (strength graph,
aggregation, prolongator smoothing, Galerkin products, dense coarse factors)
followed by the reduced solve to relative residual 1e-8 (right-hand side
K^T M_y y_d, outer CG preconditioned with the multilevel Hessian
preconditioner).  The JSON line also reports: every result's error against
the FP64 oracle's solution; the plain FP64 path, the float32-CG-in-refinement
form and the paper's comparisons (plain CG, two Hessian levels) on the same
input; 16 desired states in one batch at 64^3 and at 128^3 (2,146,689 nodes,
variance 2, beta = 1e-4); the V-cycle and the dominant kernel against the HBM
roofline; the cost of a grid barrier against a kernel boundary; and the CPU
oracle's whole step (setup + solve) timed on this host.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0

# The kernel with the largest summed device time inside the headline solves,
# read from the kernel trace of this benchmark's headline steps
# (profiles/solve_c3_kernel_trace.txt): the level-0 product of the FP64 inner
# CG (amg_time_kernel entry 4), ahead of the level-0 float32 coarse correction
# fused with the first post-smoothing step (tpro_kernel, entry 3).
DOMINANT = "cg_product"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def counter_traffic(name):
    """HBM bytes per launch of a timed kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (means over its timing loop's launches), scaled
    by the same counters' reading of a plain 256 MiB copy; None once the kernel
    sources (the kernels, their launches, or the setup that lays out their
    data) have changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{name}_hbm_counters.json")
    if not os.path.exists(path):
        return None
    m = json.load(open(path))
    h = hashlib.sha256()
    for f in ("kernels.hpp", "solver.hpp", "setup.hip"):
        h.update(open(os.path.join(ROOT, "paper_2001_11533_amd", "csrc", f), "rb").read())
    if h.hexdigest() != m.get("sources_sha256"):
        return None
    return 1024.0 * (m["fetch_kib_mean"] * m["fetch_scale"] + m["write_kib_mean"] * m["write_scale"])


def cpu_oracle(p):
    """The oracle, untuned, on the same workload: its whole step (setup of the
    hierarchy from the assembled matrices, then the reduced solve to 1e-8 with
    the GPU step's smoother) on one thread.  Then, untimed, the reference
    solution the GPU results are compared with: the same oracle solved to 1e-11."""
    from threadpoolctl import threadpool_limits

    from oracle import fem, sa, solve

    with threadpool_limits(limits=1):
        A, M = fem.assemble(p.mesh.coords, p.mesh.elems, p.kappa)
        bc = p.dirichlet.astype(bool)
        t0 = time.perf_counter()
        A0 = fem.dirichlet_stiffness(A, bc)
        h = sa.build(A0, M, bc, sa.Opts(beta=p.beta, smoother=1))
        t_setup = time.perf_counter() - t0
        o = solve.Oracle(h)
        t0 = time.perf_counter()
        u8, it8 = o.reduced_solve(p.yd[:, 0], rtol=1e-8)
        t_solve = time.perf_counter() - t0
    model, avail = host_info()
    cpu = {"value": t_setup + t_solve, "unit": "s", "cores": 1, "kind": "oracle",
           "sample": (f"the whole step of the oracle (NumPy/SciPy, FP64, one thread) on the 64^3 workload: "
                      f"setup {t_setup:.2f} s + reduced solve to 1e-8 {t_solve:.2f} s ({it8} outer iterations, "
                      f"{o.cnt.inner_iters} inner), timed once"),
           "cpu_model": model, "host_cores_available": avail}
    t0 = time.perf_counter()
    uref, itref = solve.Oracle(h).reduced_solve(p.yd[:, 0], rtol=1e-11)
    log(f"[bench] oracle reference (1e-11, {itref} outer) {time.perf_counter() - t0:.1f} s")
    return cpu, uref


def big_kernels(amg, inputs, torch, dev):
    """The level-0 kernels on the 128^3 matrix (N = 2,146,689): time per launch
    over 50 back-to-back launches with HIP events, algorithmic bytes and their
    fraction of the HBM peak."""
    p5 = inputs.config("c5", nb=16)
    rp5, ci5, va5, vm5 = amg.assemble_p1(p5.mesh.coords, p5.mesh.elems, p5.kappa)
    A5 = tuple(torch.as_tensor(x).to(dev) for x in (rp5, ci5, va5))
    M5 = tuple(torch.as_tensor(x).to(dev) for x in (rp5, ci5, vm5))
    mk5 = torch.as_tensor(p5.dirichlet).to(dev)
    del rp5, ci5, va5, vm5
    s5 = amg.HessianSolver(A5, M5, mk5, beta=p5.beta, inner_precision=32, smoother=1, autotune=1)
    big = {}
    for key, which, prec in (("presweep_f32", 1, 32), ("presweep_f64", 1, 64), ("spmv_f32", 0, 32),
                             ("tpro_f32", 3, 32), ("cg_product_f64", 4, 64), ("vcycle_f32", 2, 32)):
        ms5, by5 = s5.time_kernel(which, prec=prec, nb=1, reps=50)
        big[key] = {"us": ms5 * 1e3, "MB": by5 / 1e6, "GBps": by5 / (ms5 * 1e-3) / 1e9,
                    "frac": by5 / (ms5 * 1e-3) / 1e9 / HBM_PEAK_GBS}
    s5.close()
    return big


def run_c5(amg, inputs, torch, dev, tune_path, compare_untuned):
    """The 128^3 workload's 16 desired states in one batched solve: setup and
    solve timed with HIP events (inputs resident in HBM), with the autotuner's
    geometry for this hierarchy's products (tuned first, outside the timed
    region) and, if asked, once more with the fixed geometry rule."""
    p5 = inputs.config("c5", nb=16)
    rp5, ci5, va5, vm5 = amg.assemble_p1(p5.mesh.coords, p5.mesh.elems, p5.kappa)
    A5 = tuple(torch.as_tensor(x).to(dev) for x in (rp5, ci5, va5))
    M5 = tuple(torch.as_tensor(x).to(dev) for x in (rp5, ci5, vm5))
    mk5 = torch.as_tensor(p5.dirichlet).to(dev)
    Y5 = torch.as_tensor(p5.yd).to(dev).contiguous()
    del rp5, ci5, va5, vm5
    torch.cuda.synchronize()
    # two Hessian levels: at beta = 1e-4 the multilevel preconditioner of this
    # hierarchy is indefinite with three or more (B_0 H_0 has negative
    # eigenvalues even with tight inner solves), definite with two
    kw = dict(beta=p5.beta, inner_precision=32, smoother=1, nb_max=16, hess_levels=2)
    st = amg.HessianSolver(A5, M5, mk5, **kw)
    n_tuned = st.autotune(reps=10, cache_path=tune_path)
    st.close()

    def timed(autotune):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        s = amg.HessianSolver(A5, M5, mk5, autotune=autotune, **kw)
        ev[1].record()
        U, info = s.reduced_solve(Y5, rtol=1e-8)
        ev[2].record()
        torch.cuda.synchronize()
        return s, info, ev

    untuned_ms = None
    if compare_untuned:
        su, _, evu = timed(0)
        untuned_ms = evu[1].elapsed_time(evu[2])
        su.close()
    s5, info5, ev = timed(1)
    L5, ell5 = s5.levels()
    c5 = {"workload": "3D unit cube 128^3 Kuhn tets, N=2146689, log-normal kappa var 2, beta=1e-4, "
                      "16 bump y_d in one batch, float32 V-cycles in FP64 CG",
          "setup_ms": ev[0].elapsed_time(ev[1]), "solve_ms": ev[1].elapsed_time(ev[2]),
          "ms_per_state": ev[1].elapsed_time(ev[2]) / 16, "levels": [s5.level_size(j)[0] for j in range(L5)],
          "ell": ell5, "ell_reason": ("B_0 H_0 is indefinite with 3 or more Hessian levels at beta = 1e-4 "
                                      "(Lanczos estimate), definite with 2"),
          "outer_iters": max(i["outer_iters"] for i in info5),
          "inner_iters_total": info5[0]["inner_iters_total"], "mass_iters_total": info5[0]["mass_iters_total"],
          "solve_phase_ms": info5[0]["ms_phase"], "max_rel_resid": max(i["rel_resid"] for i in info5),
          "autotune_products_timed": n_tuned, "untuned_geometry_solve_ms": untuned_ms}
    s5.close()
    log(f"[bench] 128^3 x 16: setup {c5['setup_ms']:.0f} ms, solve {c5['solve_ms']:.0f} ms "
        f"({c5['ms_per_state']:.0f} ms per state), ell {ell5}, outer {c5['outer_iters']}, "
        f"fixed geometry rule {untuned_ms} ms")
    return c5


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-c5", action="store_true", help="skip the 128^3 batched solve")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON table of the autotuner: read first if present (its entries are not re-timed), "
                         "written back at the end of tuning")
    ap.add_argument("--c5-only", action="store_true",
                    help="only the 128^3 batch of 16 desired states (setup + solve), for its kernel statistics")
    ap.add_argument("--kernels-128-only", action="store_true",
                    help="only the level-0 kernel timings on the 128^3 matrix and the copy that calibrates the "
                         "profiler's counters (for counter runs)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline steps, the level-0 kernel timings and the copy that calibrates the "
                         "profiler's counters (for kernel traces and counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the reduced-Hessian solve of this library is a single-GPU "
              "path (independent desired states would shard by columns, one hierarchy replica per GPU; "
              "that mode is not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import inputs
    import paper_2001_11533_amd as amg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    p = inputs.config("c3")
    N = p.mesh.nverts
    log(f"[bench] workload 64^3: N={N} elements={p.mesh.nelems}")
    t0 = time.perf_counter()
    rp, ci, va, vm = amg.assemble_p1(p.mesh.coords, p.mesh.elems, p.kappa)
    host_asm_ms = (time.perf_counter() - t0) * 1e3
    # the same assembly on the GPU from device mesh arrays (outside the step: the
    # step starts from assembled matrices); wall clock per call, temporaries included
    cd = torch.as_tensor(p.mesh.coords).to(dev)
    ed = torch.as_tensor(np.ascontiguousarray(p.mesh.elems, dtype=np.int32)).to(dev)
    kd = torch.as_tensor(p.kappa).to(dev)
    got = amg.assemble_p1_device(cd, ed, kd)
    asm_same = all(np.array_equal(g.cpu().numpy(), h) for g, h in zip(got, (rp, ci, va, vm)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        got = amg.assemble_p1_device(cd, ed, kd)
    torch.cuda.synchronize()
    gpu_asm_ms = (time.perf_counter() - t0) / 5 * 1e3
    del got, cd, ed, kd
    log(f"[bench] P1 assembly 64^3: host {host_asm_ms:.1f} ms, GPU {gpu_asm_ms:.2f} ms, bit-identical {asm_same}")
    A = tuple(torch.as_tensor(x).to(dev) for x in (rp, ci, va))
    M = tuple(torch.as_tensor(x).to(dev) for x in (rp, ci, vm))
    mask = torch.as_tensor(p.dirichlet).to(dev)
    yd = torch.as_tensor(p.yd[:, 0].copy()).to(dev)
    torch.cuda.synchronize()

    tune_path = args.tune_cache or os.path.join(tempfile.mkdtemp(), "tune.json")
    if args.kernels_128_only:
        big = big_kernels(amg, inputs, torch, dev)
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"metric": "level-0 kernels on the 128^3 matrix (counter runs)", "roofline_128cube": big}),
              flush=True)
        return
    if args.c5_only:
        c5 = run_c5(amg, inputs, torch, dev, tune_path, False)
        print(json.dumps({"metric": "reduced-Hessian batched solve, 3D 128^3 P1, 16 desired states",
                          "value": c5["solve_ms"] / 1000.0, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
                          "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
                          "data": "synthetic", "config": {"workload": c5["workload"]}, "c5_batch16_128cube": c5}),
              flush=True)
        return

    def step(prec, ydv, nb_max=1, AA=None, MM=None, mk=None, beta=None, **kw):
        kw.setdefault("smoother", 1)  # V-cycles with the degree-2 Chebyshev smoother
        kw.setdefault("autotune", 1)  # the autotuner's sparse-product geometry
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        s = amg.HessianSolver(AA or A, MM or M, mask if mk is None else mk, beta=beta or p.beta,
                              inner_precision=prec, nb_max=nb_max, **kw)
        ev[1].record()
        u, info = s.reduced_solve(ydv, rtol=1e-8)
        ev[2].record()
        return s, u, info, ev

    # ---- autotuning (once per process; its table serves every later context) ----
    tuned = {}
    for nbw in (1, 16):
        s = amg.HessianSolver(A, M, mask, beta=p.beta, inner_precision=32, smoother=1, nb_max=nbw)
        tuned[nbw] = s.autotune(reps=20, cache_path=tune_path)
        s.close()
    tune_table = json.load(open(tune_path))["entries"]
    log(f"[bench] autotuner: {tuned} products timed")

    # ---- the headline step: FP32 inner / FP64 outer ----
    for _ in range(args.warmup):
        s, u, info, ev = step(32, yd)
        s.close()
    torch.cuda.synchronize()
    setup_ms, solve_ms = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        s, u, info, ev = step(32, yd)
        if k < args.steps - 1:
            s.close()
        torch.cuda.synchronize()
        setup_ms.append(ev[0].elapsed_time(ev[1]))
        solve_ms.append(ev[1].elapsed_time(ev[2]))
        log(f"[bench] step {k}: setup {setup_ms[-1]:.1f} ms solve {solve_ms[-1]:.1f} ms outer {info[0]['outer_iters']}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1000.0 * wall / args.steps
    u32 = u.clone()
    info32 = info[0]
    L, ell = s.levels()
    sizes = [s.level_size(j) for j in range(L)]
    if args.headline_only:
        for which, prec, reps in ((4, 64, 200), (3, 32, 200), (1, 32, 200), (5, 64, 200), (6, 64, 200)):
            s.time_kernel(which, prec=prec, nb=1, reps=reps)
        s.close()
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"metric": "reduced-Hessian solve time to 1e-8 (setup + solve), 3D 64^3 P1, FP32 inner / "
                                    "FP64 outer", "value": ms_step / 1000.0, "unit": "s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
                          "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
                          "data": "synthetic", "config": {"workload": "3D unit cube 64^3 Kuhn tets (headline only)"},
                          "setup_ms": float(np.median(setup_ms)), "solve_ms": float(np.median(solve_ms))}),
              flush=True)
        return
    # one more solve with the true residual and the per-phase device times
    s2 = amg.HessianSolver(A, M, mask, beta=p.beta, inner_precision=32, smoother=1, autotune=1, true_resid=1)
    _, info_tr = s2.reduced_solve(yd, rtol=1e-8)
    s2.close()

    # kernels on the library's stream (HIP events): the level-0 CG product, the
    # fused coarse correction (pass over T = A S), the pre-sweep residual, the
    # whole V-cycle; a grid barrier against a kernel boundary
    cgp_ms, cgp_bytes = s.time_kernel(4, prec=64, nb=1, reps=200)
    tpro_ms, _ = s.time_kernel(3, prec=32, nb=1, reps=200)
    pre_ms, pre_bytes = s.time_kernel(1, prec=32, nb=1, reps=200)
    vc_ms, vc_bytes = s.time_kernel(2, prec=32, nb=1, reps=50)
    bar_ms, _ = s.time_kernel(5, prec=64, nb=1, reps=200)
    bnd_ms, _ = s.time_kernel(6, prec=64, nb=1, reps=200)
    # the hierarchy's approximation numbers a~_j (Section 4), power method from a seeded vector
    gen = torch.Generator(device="cpu").manual_seed(31)
    quality = [s.hierarchy_quality(j, torch.randn(sizes[j][0], generator=gen, dtype=torch.float64).to(dev), 20)
               for j in range(L - 1)]
    log(f"[bench] a~_j: {', '.join(f'{a:.3e}' for a in quality)}")
    s.close()
    # algorithmic bytes of the method's own work (section 8(d) of the scope: int32
    # columns, vectors once): the CG product is q = A_0 p in FP64; the fused pass does
    # the prolongation S_0 e and one smoothing sweep on A_0 in float32
    n, nnzA, nnzS, _ = sizes[0]
    n1 = sizes[1][0]
    tpro_bytes = (4.0 * (n + 1) + 8.0 * nnzS + 8.0 * n + 4.0 * n1) + (4.0 * (n + 1) + 8.0 * nnzA + 8.0 * n + 12.0 * n)

    # ---- plain FP64 path, and its V-cycle ----
    s64, u64, info64, ev = step(64, yd)
    torch.cuda.synchronize()
    fp64_setup_ms, fp64_solve_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    vc64_ms, vc64_bytes = s64.time_kernel(2, prec=64, nb=1, reps=50)
    s64.close()
    log(f"[bench] fp64: setup {fp64_setup_ms:.1f} ms solve {fp64_solve_ms:.1f} ms")
    # the headline step with the fixed geometry rule instead of the autotuner's
    su, _, _, ev = step(32, yd, autotune=0)
    torch.cuda.synchronize()
    untuned_solve_ms = ev[1].elapsed_time(ev[2])
    su.close()

    # ---- the other float32 form: float32 CG inside FP64 refinement ----
    sr, ur, infor, ev = step(32, yd, mixed_mode=1)
    torch.cuda.synchronize()
    ref_solve_ms = ev[1].elapsed_time(ev[2])
    sr.close()
    log(f"[bench] fp32 refinement form: solve {ref_solve_ms:.1f} ms")

    # ---- the paper's comparisons on this workload: plain outer CG (Table 4's
    # setting) and two Hessian levels (Table 5's), same inner solves; and the
    # V-cycle with one l1-Jacobi sweep instead of the Chebyshev smoother ----
    variants, var_u = {}, {}
    for key, kw in (("plain_cg", {"precond": 0}), ("two_level", {"hess_levels": 2}),
                    ("l1_jacobi_smoother", {"smoother": 0})):
        sv, uv, infov, ev = step(32, yd, **kw)
        torch.cuda.synchronize()
        variants[key] = {"outer_iters": infov[0]["outer_iters"], "solve_ms": ev[1].elapsed_time(ev[2]),
                         "inner_iters_total": infov[0]["inner_iters_total"]}
        var_u[key] = uv.clone()
        sv.close()
        log(f"[bench] {key}: outer {variants[key]['outer_iters']} solve {variants[key]['solve_ms']:.1f} ms")

    # ---- 16 desired states as one block solve (column 0 is the headline's y_d) ----
    yd16 = torch.as_tensor(inputs.config("c3", nb=16).yd).to(dev).contiguous()
    sb, ub, infob, ev = step(32, yd16, nb_max=16)
    torch.cuda.synchronize()
    batch_solve_ms = ev[1].elapsed_time(ev[2])
    sb.close()
    # the same batch with the fixed geometry rule instead of the autotuner's
    sbu, _, _, ev = step(32, yd16, nb_max=16, autotune=0)
    torch.cuda.synchronize()
    batch_untuned_ms = ev[1].elapsed_time(ev[2])
    sbu.close()
    log(f"[bench] batch16 solve {batch_solve_ms:.1f} ms ({batch_solve_ms / 16:.1f} ms per state), "
        f"fixed geometry rule {batch_untuned_ms:.1f} ms")

    # ---- the same kernels on the 128^3 level-0 matrix (N = 2,146,689, 263 MB
    # float32): past the caches, where launch overheads no longer dominate; and
    # the 128^3 workload's 16 desired states in one batched solve ----
    big = big_kernels(amg, inputs, torch, dev)
    log(f"[bench] 128^3 level 0: pre-sweep f32 {big['presweep_f32']['GBps']:.0f} GB/s, "
        f"CG product f64 {big['cg_product_f64']['GBps']:.0f} GB/s")
    c5 = None if args.no_c5 else run_c5(amg, inputs, torch, dev, tune_path, True)

    # ---- a plain device copy of 256 MiB: the reference that scales the
    # rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes ----
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    # ---- the CPU oracle: its whole step timed, and the reference solution ----
    cpu, uref = cpu_oracle(p)
    log(f"[bench] cpu oracle step {cpu['value']:.1f} s")

    def err(x):
        x = x.detach().cpu().numpy().reshape(-1) if hasattr(x, "detach") else np.asarray(x)
        return float(np.linalg.norm(x - uref) / np.linalg.norm(uref))

    errors = {"headline_fp32_preconditioned": err(u32), "fp64": err(u64), "fp32_refinement": err(ur),
              "plain_cg": err(var_u["plain_cg"]), "two_level": err(var_u["two_level"]),
              "l1_jacobi_smoother": err(var_u["l1_jacobi_smoother"]), "batch16_column0": err(ub[:, 0])}
    log(f"[bench] errors vs oracle: {errors}")

    rooflines = {
        "cg_product": {"bound": "hbm", "achieved": cgp_bytes / (cgp_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": cgp_bytes / (cgp_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "traffic": counter_traffic("cg_product_c3"),
                       "kernel": ("level-0 product of the FP64 inner CG preconditioned by float32 V-cycles, "
                                  "q = A_0 z + beta q_old with the previous iteration's finalize folded in "
                                  "(sell_kernel<double,1,GZ<double,1,float>,ECgQR<double,1,float>,FusedFin<1,false>>)"),
                       "ms": cgp_ms, "bytes": cgp_bytes,
                       "bytes_rule": "4(n+1) + (4+8) nnz(A_0) + 2*8 n: the method's q = A_0 p, FP64, int32 columns",
                       "timing": ("HIP events on the library stream over 200 back-to-back launches that rotate "
                                  "the slice-to-XCD assignment, so no launch reuses its L2")},
        "tpro": {"bound": "hbm", "achieved": tpro_bytes / (tpro_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": tpro_bytes / (tpro_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "traffic": counter_traffic("tpro_cheb_c3"),
                 "kernel": ("level-0 float32 coarse correction fused with the first post-smoothing step, "
                            "one pass over T = A S (tpro_kernel<float,1,0,EProCheb>)"),
                 "ms": tpro_ms, "bytes": tpro_bytes,
                 "bytes_rule": ("the method's work it does: prolongation S_0 e (4(n+1) + 8 nnz(S_0) + 2*4 n + 4 n_1) "
                                "and one smoothing sweep on A_0 (4(n+1) + 8 nnz(A_0) + 2*4 n + 3*4 n), float32"),
                 "timing": "HIP events on the library stream over 200 back-to-back launches"},
        "presweep": {"bound": "hbm", "achieved": pre_bytes / (pre_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": pre_bytes / (pre_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": counter_traffic("sell_presweep_c3"),
                     "kernel": ("level-0 float32 pre-sweep residual r = b - A x of the V-cycle "
                                "(sell_kernel<float,0,GPlain,EResB>)"),
                     "ms": pre_ms, "bytes": pre_bytes,
                     "bytes_rule": ("4(n+1) + (2+4) nnz(A_0) + 3*4 n: r = b - A_0 x, float32, counted with the 16-bit "
                                    "column offsets the sliced-ELL level-0 matrix stores (int32 columns: 33.8 MB)"),
                     "timing": ("HIP events on the library stream over 200 back-to-back launches that rotate "
                                "the slice-to-XCD assignment, so no launch reuses its L2")},
    }
    res = {
        "metric": "reduced-Hessian solve time to 1e-8 (setup + solve), 3D 64^3 P1, FP32 inner / FP64 outer",
        "value": ms_step / 1000.0,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "3D unit cube 64^3 Kuhn tets, P1, N=274625, log-normal kappa var 1, beta=1e-3, "
                               "eq. test-state y_d, nb=1", "N": N, "levels": sizes, "ell": ell,
                   "inner": "FP64 CG preconditioned by float32 V-cycles",
                   "smoother": "Chebyshev degree 2 on the l1 diagonal",
                   "geometry": "autotuned (amg_autotune, process-wide table)"},
        "setup_ms": float(np.median(setup_ms)),
        "solve_ms": float(np.median(solve_ms)),
        "outer_iters": info32["outer_iters"],
        "inner_solves": info32["inner_solves"],
        "inner_iters_total": info32["inner_iters_total"],
        "rel_resid": info32["rel_resid"],
        "true_rel_resid": info_tr[0]["true_rel_resid"],
        "solve_phase_ms": info_tr[0]["ms_phase"],
        "solve_bytes_moved": info_tr[0]["bytes_moved"],
        "err_vs_oracle": errors,
        "fp64": {"setup_ms": fp64_setup_ms, "solve_ms": fp64_solve_ms, "outer_iters": info64[0]["outer_iters"]},
        "untuned_geometry_solve_ms": untuned_solve_ms,
        "autotune": {"products_timed": tuned, "choices": {e["key"]: e["lg"] for e in tune_table}},
        "fp32_refinement": {"solve_ms": ref_solve_ms, "outer_iters": infor[0]["outer_iters"],
                            "refine_steps": infor[0]["refine_steps"]},
        "multilevel_vs": variants,
        "hierarchy_quality_a_tilde": quality,
        "batch16": {"solve_ms": batch_solve_ms, "ms_per_state": batch_solve_ms / 16,
                    "untuned_geometry_solve_ms": batch_untuned_ms,
                    "outer_iters": max(i["outer_iters"] for i in infob)},
        "c5_batch16_128cube": c5,
        "vcycle": {"f32_ms": vc_ms, "f32_GBps_alg": vc_bytes / (vc_ms * 1e-3) / 1e9,
                   "f64_ms": vc64_ms, "f64_GBps_alg": vc64_bytes / (vc64_ms * 1e-3) / 1e9},
        "roofline": dict(rooflines[DOMINANT], dominant=("largest summed device time in the headline solve's "
                                                        "kernel trace (profiles/solve_c3_kernel_trace.txt)")),
        "roofline_others": {k: v for k, v in rooflines.items() if k != DOMINANT},
        "roofline_128cube": dict(big, note="the same kernels on the 128^3 level-0 matrix, algorithmic bytes"),
        "grid_sync_us": {"cooperative_grid_barrier": bar_ms * 1e3, "kernel_boundary": bnd_ms * 1e3,
                         "note": ("one workgroup per CU, an elementwise step over 2^16 floats per round; "
                                  "barrier = release fence, arrival counter, generation flag, acquire fence")},
        "assembly_64cube": {"host_ms": host_asm_ms, "gpu_ms": gpu_asm_ms, "bit_identical": asm_same,
                            "note": "P1 stiffness and mass of the 64^3 mesh, outside the timed step"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
