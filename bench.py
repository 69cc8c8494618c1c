"""Benchmark of the reduced-Hessian solve on one MI355X.

Workload: the 3D unit cube, 64^3 grid split into 6 Kuhn tetrahedra per cube
(274,625 nodes, 1,572,864 P1 elements), log-normal kappa (16 seeded Fourier
modes, variance 1), beta = 1e-3, the manufactured desired state of the paper's
eq. test-state; inner A-solves by FP64 CG preconditioned with float32
V-cycles (the bulk of the traffic; degree-2 Chebyshev smoothing on the l1
diagonal), outer Hessian CG, CG residuals, dot products and dense coarse
factors in FP64.

One step = the whole hot path on that input, resident in HBM when the timed
region starts: the smoothed-aggregation setup on the GPU (strength graph,
aggregation, prolongator smoothing, Galerkin products, dense coarse factors)
followed by the reduced solve to relative residual 1e-8 (right-hand side
K^T M_y y_d, outer CG preconditioned with the multilevel Hessian
preconditioner).  The JSON line also reports the plain FP64 path, the
float32-CG-in-refinement form, the batched
(16 desired states) path, the V-cycle and dominant-kernel bandwidth, and the
CPU oracle timed on a bounded sample on this host.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counter_traffic(name="sell_presweep_c3"):
    """HBM bytes per launch of a timed kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (means over its timing loop's launches), scaled
    by the same counters' reading of a plain 256 MiB copy; None once the kernel
    source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{name}_hbm_counters.json")
    if not os.path.exists(path):
        return None
    m = json.load(open(path))
    src = os.path.join(ROOT, "paper_2001_11533_amd", "csrc", "kernels.hpp")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m["kernels_hpp_sha256"]:
        return None
    return 1024.0 * (m["fetch_kib_mean"] * m["fetch_scale"] + m["write_kib_mean"] * m["write_scale"])


def cpu_baseline(p, gpu_outer_iters: int):
    """The oracle, untuned, on a bounded sample of the same workload: its full
    setup (hierarchy from the assembled matrices), its right-hand side and one
    outer iteration (one Hessian action and one preconditioner action), scaled
    to a whole step with the outer-iteration count of the GPU solve."""
    from threadpoolctl import threadpool_limits

    from oracle import fem, sa, solve

    with threadpool_limits(limits=1):
        A, M = fem.assemble(p.mesh.coords, p.mesh.elems, p.kappa)
        bc = p.dirichlet.astype(bool)
        t0 = time.perf_counter()
        A0 = fem.dirichlet_stiffness(A, bc)
        h = sa.build(A0, M, bc, sa.Opts(beta=p.beta, smoother=1))  # the GPU step's configuration
        t_setup = time.perf_counter() - t0
        o = solve.Oracle(h)
        t0 = time.perf_counter()
        b = o.rhs(p.yd[:, 0])
        t_rhs = time.perf_counter() - t0
        t0 = time.perf_counter()
        o.hessian_apply(0, b)
        o.precond(b)
        t_iter = time.perf_counter() - t0
    est = t_setup + t_rhs + gpu_outer_iters * t_iter + t_iter  # + the initial preconditioner/Hessian work
    return {"value": est, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle (NumPy/SciPy, FP64, 1 thread) on the 64^3 workload: full setup {t_setup:.1f} s, "
                       f"rhs {t_rhs:.1f} s, one outer iteration {t_iter:.1f} s measured; step = setup + rhs + "
                       f"({gpu_outer_iters} + 1) outer iterations")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
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

    def step(prec, ydv, nb_max=1, **kw):
        kw.setdefault("smoother", 1)  # V-cycles with the degree-2 Chebyshev smoother
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        s = amg.HessianSolver(A, M, mask, beta=p.beta, inner_precision=prec, nb_max=nb_max, **kw)
        ev[1].record()
        u, info = s.reduced_solve(ydv, rtol=1e-8)
        ev[2].record()
        return s, u, info, ev

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

    # level-0 float32 kernels and the whole V-cycle, HIP events on the library's stream:
    # the pre-sweep residual (sliced ELL) and the fused coarse correction (pass over T = A S)
    kern_ms, kern_bytes = s.time_kernel(1, prec=32, nb=1, reps=200)
    tpro_ms, tpro_bytes = s.time_kernel(3, prec=32, nb=1, reps=200)
    vc_ms, vc_bytes = s.time_kernel(2, prec=32, nb=1, reps=50)
    vc64_ms = vc64_bytes = None
    # the hierarchy's approximation numbers a~_j (Section 4), power method from a seeded vector
    gen = torch.Generator(device="cpu").manual_seed(31)
    quality = [s.hierarchy_quality(j, torch.randn(sizes[j][0], generator=gen, dtype=torch.float64).to(dev), 20)
               for j in range(L - 1)]
    log(f"[bench] a~_j: {', '.join(f'{a:.3e}' for a in quality)}")
    s.close()

    # ---- plain FP64 path on the same input ----
    s64, u64, info64, ev = step(64, yd)
    torch.cuda.synchronize()
    fp64_setup_ms, fp64_solve_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    err_mixed_vs_fp64 = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
    vc64_ms, vc64_bytes = s64.time_kernel(2, prec=64, nb=1, reps=50)
    s64.close()
    log(f"[bench] fp64: setup {fp64_setup_ms:.1f} ms solve {fp64_solve_ms:.1f} ms; mixed vs fp64 {err_mixed_vs_fp64:.2e}")

    # ---- the other float32 form: float32 CG inside FP64 refinement ----
    sr, ur, infor, ev = step(32, yd, mixed_mode=1)
    torch.cuda.synchronize()
    ref_solve_ms = ev[1].elapsed_time(ev[2])
    err_refine_vs_fp64 = float(torch.linalg.norm(ur - u64) / torch.linalg.norm(u64))
    sr.close()
    log(f"[bench] fp32 refinement form: solve {ref_solve_ms:.1f} ms; vs fp64 {err_refine_vs_fp64:.2e}")

    # ---- the paper's comparisons on this workload: plain outer CG (Table 4's
    # setting) and two Hessian levels (Table 5's), same inner solves; and the
    # V-cycle with one l1-Jacobi sweep instead of the Chebyshev smoother ----
    variants = {}
    for key, kw in (("plain_cg", {"precond": 0}), ("two_level", {"hess_levels": 2}),
                    ("l1_jacobi_smoother", {"smoother": 0})):
        sv, uv, infov, ev = step(32, yd, **kw)
        torch.cuda.synchronize()
        variants[key] = {"outer_iters": infov[0]["outer_iters"], "solve_ms": ev[1].elapsed_time(ev[2]),
                         "inner_iters_total": infov[0]["inner_iters_total"],
                         "rel_diff_vs_multilevel": float(torch.linalg.norm(uv - u32) / torch.linalg.norm(u32))}
        sv.close()
        log(f"[bench] {key}: outer {variants[key]['outer_iters']} solve {variants[key]['solve_ms']:.1f} ms")

    # ---- 16 desired states as one block solve vs one at a time ----
    yd16 = torch.as_tensor(inputs.config("c3", nb=16).yd).to(dev).contiguous()
    sb, ub, infob, ev = step(32, yd16, nb_max=16)
    torch.cuda.synchronize()
    batch_solve_ms = ev[1].elapsed_time(ev[2])
    sb.close()
    log(f"[bench] batch16 solve {batch_solve_ms:.1f} ms ({batch_solve_ms / 16:.1f} ms per state)")

    # ---- the same kernels on the 128^3 level-0 matrix (N = 2,146,689, 263 MB
    # float32): past the caches, where launch overheads no longer dominate ----
    p5 = inputs.config("c5", nb=1)
    rp5, ci5, va5, vm5 = amg.assemble_p1(p5.mesh.coords, p5.mesh.elems, p5.kappa)
    s5 = amg.HessianSolver(tuple(torch.as_tensor(x).to(dev) for x in (rp5, ci5, va5)),
                           tuple(torch.as_tensor(x).to(dev) for x in (rp5, ci5, vm5)),
                           torch.as_tensor(p5.dirichlet).to(dev), beta=p5.beta, inner_precision=32, smoother=1)
    big = {}
    for key, which, prec in (("presweep_f32", 1, 32), ("presweep_f64", 1, 64), ("spmv_f32", 0, 32),
                             ("tpro_f32", 3, 32), ("vcycle_f32", 2, 32)):
        ms5, by5 = s5.time_kernel(which, prec=prec, nb=1, reps=50)
        big[key] = {"us": ms5 * 1e3, "MB": by5 / 1e6, "GBps": by5 / (ms5 * 1e-3) / 1e9,
                    "frac": by5 / (ms5 * 1e-3) / 1e9 / HBM_PEAK_GBS}
    s5.close()
    del rp5, ci5, va5, vm5
    log(f"[bench] 128^3 level 0: pre-sweep f32 {big['presweep_f32']['GBps']:.0f} GB/s, "
        f"V-cycle f32 {big['vcycle_f32']['GBps']:.0f} GB/s")

    # ---- a plain device copy of 256 MiB: the reference that scales the
    # rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes ----
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    # ---- CPU oracle on a bounded sample ----
    cpu = cpu_baseline(p, info32["outer_iters"])
    log(f"[bench] cpu baseline {cpu['value']:.1f} s")

    achieved = kern_bytes / (kern_ms * 1e-3) / 1e9
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
               "smoother": "Chebyshev degree 2 on the l1 diagonal"},
        "setup_ms": float(np.median(setup_ms)),
        "solve_ms": float(np.median(solve_ms)),
        "outer_iters": info32["outer_iters"],
        "inner_solves": info32["inner_solves"],
        "inner_iters_total": info32["inner_iters_total"],
        "refine_steps": info32["refine_steps"],
        "rel_resid": info32["rel_resid"],
        "fp64": {"setup_ms": fp64_setup_ms, "solve_ms": fp64_solve_ms, "outer_iters": info64[0]["outer_iters"]},
        "err_mixed_vs_fp64": err_mixed_vs_fp64,
        "fp32_refinement": {"solve_ms": ref_solve_ms, "outer_iters": infor[0]["outer_iters"],
                            "refine_steps": infor[0]["refine_steps"], "err_vs_fp64": err_refine_vs_fp64},
        "multilevel_vs": variants,
        "hierarchy_quality_a_tilde": quality,
        "batch16": {"solve_ms": batch_solve_ms, "ms_per_state": batch_solve_ms / 16,
                    "outer_iters": max(i["outer_iters"] for i in infob)},
        "vcycle": {"f32_ms": vc_ms, "f32_GBps_alg": vc_bytes / (vc_ms * 1e-3) / 1e9,
                   "f64_ms": vc64_ms, "f64_GBps_alg": vc64_bytes / (vc64_ms * 1e-3) / 1e9},
        "roofline": {"bound": "hbm", "achieved": tpro_bytes / (tpro_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": tpro_bytes / (tpro_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": counter_traffic("tpro_cheb_c3"),
                     "kernel": ("level-0 float32 coarse correction fused with the first post-smoothing step, "
                                "one pass over T = A S (tpro_kernel<float,1,0,EProCheb>)"),
                     "ms": tpro_ms, "bytes": tpro_bytes,
                     "timing": "HIP events on the library stream over 200 back-to-back launches"},
        "roofline_presweep": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic("sell_presweep_c3"),
                              "kernel": ("level-0 float32 pre-sweep residual r = b - A x of the V-cycle "
                                         "(sell_kernel<float,0,GPlain,EResB>)"),
                              "ms": kern_ms, "bytes": kern_bytes,
                              "timing": ("HIP events on the library stream over 200 back-to-back launches that "
                                         "rotate the slice-to-XCD assignment, so no launch reuses its L2")},
        "roofline_128cube": dict(big, note="same kernels on the 128^3 level-0 matrix, timed as in "
                                           "roofline; algorithmic bytes as in roofline"),
        "assembly_64cube": {"host_ms": host_asm_ms, "gpu_ms": gpu_asm_ms, "bit_identical": asm_same,
                            "note": "P1 stiffness and mass of the 64^3 mesh, outside the timed step"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
