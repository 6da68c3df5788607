"""Benchmark: 256^3 elastic Helmholtz solves per second, float32-preconditioned
vs float64, and the stencil apply's HBM bandwidth.

Workload (default): 3D 256^3 grid, layered synthetic medium from seed 3
(Vp in [1.5, 4.5] with Gaussian perturbations, Vs = Vp/1.73,
rho = 0.25 + 0.5 Vp), h = 1, 10 points per minimal shear wavelength,
gamma = 0.01, absorbing layer of 16 cells, one point source (u_3 at the
centre face); beta = 2/3; flexible GMRES(5) in float64 to a 1e-6 relative
residual, right-preconditioned by 4-level K(1,1)-cycles on the shifted operator (alpha = 0.5; each
level's two coarse calls precondition two flexible-GCR steps; damping 0.6/0.5/0.4/0.4; coarsest solve
GMRES with a budget of 2 preconditioned by one Vanka sweep; V and W cycles with --cycle V / W).
One step = one complete solve from a zero initial guess.  The headline
value is the solve rate with the float32 cycle; the same solve with the
float64 cycle is timed beside it.

Prints ONE JSON line (rank 0).  `python bench.py --gpus N` with N > 1 exits:
the library and this benchmark run on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E peak, GB/s
APPLY_BYTES_F64 = 152      # algorithmic bytes per cell of one operator apply (x, y, mu, rho, kappa)
APPLY_BYTES_F32 = 76
RESID_BYTES_F32 = 108      # residual b - H_s x in complex64: x, b, y (32 B each) + mu, rho, kappa (float32)
# HBM bytes per launch of the float32 residual at 256^3 from the rocprofv3
# FETCH_SIZE / WRITE_SIZE passes over `bench.py --pmc-target`
# (profiles/stencil_256cubed_counters.md; FETCH_SIZE x2.0, WRITE_SIZE x1.0):
# 1.822 GB read + 0.563 GB written, measured on the kernel source whose
# SHA-256 prefix is RESID_TRAFFIC_SOURCE.  When the source changes the
# figure is not reported (null) until the passes are repeated.
RESID_TRAFFIC_BYTES = 2.385e9
RESID_TRAFFIC_SOURCE = "0668f9b40eca824f"
STENCIL_SOURCE = os.path.join(ROOT, "paper_2307_03242_amd", "csrc", "elh_stencil3d_wave.hip")


def stencil_source_hash():
    import hashlib
    with open(STENCIL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--alpha", type=float, default=0.5)
    ap.add_argument("--damping", type=str, default="0.6,0.5,0.4,0.4")
    ap.add_argument("--abl", type=int, default=16, help="absorbing layer width in cells")
    ap.add_argument("--coarse", type=str, default="krylov")
    ap.add_argument("--cycle", type=str, default="K", choices=["V", "W", "K"])
    ap.add_argument("--coarse-sweeps", type=int, default=1)
    ap.add_argument("--coarse-maxit", type=int, default=2)
    ap.add_argument("--coarse-rtol", type=float, default=0.0)
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--maxit", type=int, default=400)
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=64, help="oracle sample grid (cells per axis)")
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--pmc-target", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration) and, at --n^3 in complex64, the "
                         "residual, the apply, a Vanka half-sweep (residual + block solves) and the fused residual "
                         "restriction, each after one untimed call (which lets the autotuner choose) and then three "
                         "times, for rocprofv3 --pmc passes")
    ap.add_argument("--paper-tables", action="store_true",
                    help="only the 2D iteration-count experiments of the paper's homogeneous and linear-media "
                         "tables (W(1,1) cycles, 2-4 levels, beta 1 and 2/3), counts beside the printed ones")
    ap.add_argument("--paper-3d", action="store_true",
                    help="only the 3D iteration counts on the paper's Overthrust grid shapes (synthetic layered "
                         "media stand in for the model), beside the printed ones")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-sources, uneven-batch and gradient measurements")
    return ap.parse_args()


def cpu_baseline(args, gpu_iters, cfg):
    """Oracle (plain NumPy/SciPy float64) on the host: the same solver on a
    --cpu-n^3 grid of the same media recipe, timed over --cpu-iters outer
    FGMRES iterations (hierarchy setup excluded), scaled per cell to the
    benchmark grid and multiplied by the GPU's iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import grid as G, operator as O, cycle as C
    from oracle.krylov import fgmres
    from synthetic import make_media, point_source, omega_for_ppw, random_field
    n = args.cpu_n
    shape = (n, n, n)
    m = make_media(shape, args.seed)
    om = omega_for_ppw(m["vs"].min(), 1.0, 10)
    lv = G.Level(shape, 1.0, om, 0.01, 2 / 3, m["lam"], m["mu"], m["rho"],
                 abl_width=args.abl * n / args.n, abl_amp=2.0)
    with threadpool_limits(limits=1):
        hier = C.Hierarchy(lv, C.CycleParams(levels=args.levels, alpha=args.alpha,
                                             damping=cfg["damping"], coarse=args.coarse,
                                             coarse_sweeps=args.coarse_sweeps,
                                             coarse_maxit=args.coarse_maxit, coarse_rtol=args.coarse_rtol,
                                             calls={"V": 1, "W": 2, "K": 3}[args.cycle]))
        A = O.assemble(lv)
        b = G.pack(lv, point_source(shape))
        t0 = time.perf_counter()
        _, info = fgmres(lambda v: A @ v, b, precond=hier.vcycle, restart=5, tol=0.0,
                         maxit=args.cpu_iters)
        dt = time.perf_counter() - t0
    per_iter_cell = dt / info["iters"] / (n ** 3)
    t_solve = per_iter_cell * (args.n ** 3) * gpu_iters
    # the oracle's matrix-free apply, measured at full sizes (one core)
    applies = {}
    for na in (128, args.n):
        if na in applies or na <= 0:
            continue
        ma = make_media((na, na, na), args.seed)
        la = G.Level((na, na, na), 1.0, omega_for_ppw(ma["vs"].min(), 1.0, 10), 0.01, 2 / 3, ma["lam"], ma["mu"],
                     ma["rho"], abl_width=args.abl * 1.0, abl_amp=2.0)
        xa = random_field((na, na, na), 1)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            ya = O.apply(la, xa)
            ta = time.perf_counter() - t0
        applies["%d^3" % na] = {"seconds": ta, "GBps": APPLY_BYTES_F64 * na ** 3 / ta / 1e9}
        del ma, la, xa, ya
    cpu_model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "%d outer FGMRES(5)+%s-cycle iterations of the float64 oracle on a %d^3 grid "
                      "(same media recipe, %.1f s), scaled per cell to %d^3 and to the GPU's %d iterations"
                      % (info["iters"], args.cycle, n, dt, args.n, gpu_iters),
            "cpu_model": cpu_model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "oracle_apply_measured": applies}


def solver_cfg(args, omega, levels=None):
    damping = [float(v) for v in args.damping.split(",")]
    return dict(h=1.0, omega=omega, gamma=0.01, alpha=args.alpha, beta=2 / 3, abl_width=args.abl * 1.0,
                abl_amp=2.0, levels=levels or args.levels, nu1=1, nu2=1, cycle=args.cycle, damping=damping,
                coarse_mode=args.coarse, coarse_sweeps=args.coarse_sweeps, coarse_restart=5,
                coarse_maxit=args.coarse_maxit, coarse_rtol=args.coarse_rtol)


def extras(args):
    """Secondary measurements of the other production forms (one run each,
    setup excluded): batched sources, uneven-grid batch, FWI gradient."""
    import os
    import torch
    from paper_2307_03242_amd import Problem
    from paper_2307_03242_amd.autograd import misfit
    from synthetic import make_media, point_source, omega_for_ppw, lattice_sources
    out = {}

    def media(shape, seed):
        m = make_media(shape, seed)
        return m, [torch.from_numpy(m[k]).cuda() for k in ("lam", "mu", "rho")]

    # 32 point sources on a 160^3 grid: one batched float32-cycle solve vs the
    # plain float64 solver (float64 cycle, no graphs) one source at a time
    n = 160
    shape = (n, n, n)
    m, med = media(shape, 4)
    om = omega_for_ppw(m["vs"].min(), 1.0, 10)
    q = torch.from_numpy(lattice_sources(shape, 4, 8, depth_index=args.abl + 2, margin=args.abl)).cuda()
    p32 = Problem(*med, precond_dtype=torch.complex64, **solver_cfg(args, om))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info, code = p32.solve(q, rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    iters32 = [i["iters"] for i in info]
    del p32
    torch.cuda.empty_cache()
    # the plain float64 solver with the library's defaults (graphs on), one
    # source per solve, all 32 sources (after one untimed solve that tunes);
    # and the same float64 solver on the whole batch in one call
    p64 = Problem(*med, precond_dtype=torch.complex128, **solver_cfg(args, om))
    p64.solve(q[0:1].contiguous(), rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(32):
        p64.solve(q[s:s + 1].contiguous(), rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / 32
    t0 = time.perf_counter()
    _, info64b, code64b = p64.solve(q, rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    tb64 = time.perf_counter() - t0
    del p64
    torch.cuda.empty_cache()
    out["batched_sources"] = {
        "workload": "160^3, seed 4, 32 point sources (u_3, 4x8 lattice), float32 cycle, one batched solve "
                    "(converged sources leave the batch at restarts)",
        "solves_per_s": 32 / tb, "iters_min": min(iters32), "iters_max": max(iters32), "code": code,
        "baseline_fp64_single_solves_per_s": 1.0 / ts,
        "baseline": "float64 cycle, library defaults (graphs on), one source per solve, all 32 sources",
        "speedup": ts * 32 / tb,
        "fp64_batched_solves_per_s": 32 / tb64, "speedup_vs_fp64_batched": tb64 / tb, "fp64_batched_code": code64b}

    # 12 independent problems of uneven size in one batch handle (a library
    # stream each, driven side by side), against the same problems solved one
    # after another through their own handles
    from paper_2307_03242_amd import Batch
    sizes = [64, 80, 96, 112, 128, 144, 160, 176, 192, 96, 128, 160]
    specs, qs = [], []
    for i, nn in enumerate(sizes):
        sh = (nn, nn, nn)
        mm, md = media(sh, 100 + i)
        omi = omega_for_ppw(mm["vs"].min(), 1.0, 10)
        specs.append(dict(lam=md[0], mu=md[1], rho=md[2], precond_dtype=torch.complex64, **solver_cfg(args, omi)))
        qs.append(torch.from_numpy(point_source(sh)[None]).cuda())
    batch = Batch(specs)
    batch.solve(qs, rtol=args.rtol, maxit=args.maxit)   # tunes and records the graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infos, code = batch.solve(qs, rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    tc = time.perf_counter() - t0
    t0 = time.perf_counter()
    for i, qq in enumerate(qs):
        batch.problem(i).solve(qq, rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    tq = time.perf_counter() - t0
    out["uneven_batch"] = {
        "workload": "12 problems, n = %s (seeds 100-111), 1 centred source each, float32 cycle, one batch handle"
                    % sizes,
        "solves_per_s_concurrent": len(sizes) / tc, "solves_per_s_sequential": len(sizes) / tq,
        "concurrent_over_sequential": tq / tc,
        "iters": [i[0]["iters"] for i in infos], "code": code}
    batch.close()
    del batch, specs, qs
    torch.cuda.empty_cache()

    # FWI gradient on 128^3: 8 sources, receivers on the plane at depth 18
    n = 128
    shape = (n, n, n)
    mt, medt = media(shape, 500)
    om = omega_for_ppw(mt["vs"].min(), 1.0, 10)
    src = torch.from_numpy(lattice_sources(shape, 2, 4, depth_index=18, margin=args.abl)).cuda()
    mask = torch.zeros((4,) + shape, dtype=torch.bool, device="cuda")
    mask[:3, 18, args.abl:-args.abl, args.abl:-args.abl] = True
    pt = Problem(*medt, precond_dtype=torch.complex64, **solver_cfg(args, om))
    d_obs, _, _ = pt.solve(src, rtol=args.rtol, maxit=args.maxit)
    d_obs = d_obs * mask
    z, y, x = torch.meshgrid(*[torch.arange(n, dtype=torch.float64, device="cuda") + 0.5] * 3, indexing="ij")
    blob = 1.0 - 0.08 * torch.exp(-((z - n / 2) ** 2 + (y - n / 2) ** 2 + (x - n / 2) ** 2) / (2 * 12.0 ** 2))
    params = [(mm * blob).clone().requires_grad_(True) for mm in medt]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi = misfit(pt, *params, src, mask, d_obs, rtol=args.rtol, maxit=args.maxit)
    phi.backward()
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    # the paper's coarsest solver (Section 3.2: p eliminated, FGMRES(5) on the
    # Schur complement preconditioned by 10 hybrid Kaczmarz sweeps with
    # relaxation 0.8, to a residual drop of 0.1 with at most 250 sweeps) in
    # place of the default coarsest solve, same --n^3 problem and K-cycle
    n = args.n
    shape = (n, n, n)
    mk_, medk = media(shape, args.seed)
    om = omega_for_ppw(mk_["vs"].min(), 1.0, 10)
    qk = torch.from_numpy(point_source(shape)[None]).cuda()
    kz = {"workload": "%d^3, seed %d, 1 point source, float32 %d-level %s-cycle; coarsest solve: Schur complement "
                      "FGMRES(5), 10 hybrid Kaczmarz sweeps per step (relaxation 0.8), residual drop 0.1, "
                      "<= 250 sweeps" % (n, args.seed, args.levels, args.cycle)}
    for box in (2, 4):
        cfg = solver_cfg(args, om)
        cfg.update(coarse_mode="kaczmarz", coarse_sweeps=10, coarse_restart=5, coarse_maxit=25, coarse_rtol=0.1,
                   coarse_damping=0.8)
        pk = Problem(*medk, precond_dtype=torch.complex64, kacz_box=box, **cfg)
        cs, _ = pk.level_shape(args.levels - 1)
        bc = torch.ones((1, 4) + tuple(cs), dtype=torch.complex64, device="cuda")
        pk.kaczmarz(bc, 10)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            pk.kaczmarz(bc, 10)
        e1.record()
        e1.synchronize()
        pk.solve(qk, rtol=args.rtol, maxit=args.maxit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, code = pk.solve(qk, rtol=args.rtol, maxit=args.maxit)
        torch.cuda.synchronize()
        tk = time.perf_counter() - t0
        kz["box_%d" % box] = {"solves_per_s": 1.0 / tk, "iters": info[0]["iters"], "code": code,
                              "coarsest": "%dx%dx%d" % tuple(reversed(cs)),
                              "ms_per_10_sweeps": e0.elapsed_time(e1) / 10,
                              "precond_ms": info[0]["t_precond_ms"]}
        del pk
        torch.cuda.empty_cache()
    out["paper_coarsest_solver"] = kz

    out["fwi_gradient"] = {
        "workload": "128^3, true medium seed 500, start = true with an 8%% central Gaussian anomaly, 8 sources, "
                    "receivers on the plane at depth 18; forward + adjoint solves to %.0e + gradient kernel" % args.rtol,
        "seconds": tg, "misfit": float(phi.item())}

    # one GPU's share of the 256^3 grid split into x_3 slabs over 8 GPUs:
    # 256 x 256 x 32 cells plus a one-plane halo on each side, the kernels
    # at that shape (HIP events on the library's stream)
    from synthetic import random_field
    sh = (34, 256, 256)
    ms_, meds = media(sh, 3)
    ps = Problem(*meds, precond_dtype=torch.complex64, h=1.0, omega=omega_for_ppw(ms_["vs"].min(), 1.0, 10),
                 gamma=0.01, alpha=args.alpha, beta=2 / 3, abl_width=args.abl * 1.0, abl_amp=2.0, levels=2,
                 cycle="K", coarse_mode="relax", coarse_sweeps=1)
    ncell = 34 * 256 * 256
    st = torch.cuda.current_stream()

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    x32 = torch.from_numpy(random_field(sh, 1)).cuda().to(torch.complex64)
    b32 = torch.from_numpy(random_field(sh, 2)).cuda().to(torch.complex64)
    r32 = torch.empty_like(x32)
    x64 = x32.to(torch.complex128)
    y64 = torch.empty_like(x64)
    t_res = timed(lambda: ps.residual(b32, x32, shifted=True, out=r32))
    t_app = timed(lambda: ps.apply(x64, out=y64))
    t_rel = timed(lambda: ps.relax(b32, r32, 0))
    out["shard_slab"] = {
        "workload": "256 x 256 x 34 cells (one of 8 x_3 slabs of 256^3 with a one-plane halo each side), seed 3 media",
        "residual_f32_ms": t_res, "residual_f32_GBps": RESID_BYTES_F32 * ncell / (t_res * 1e-3) / 1e9,
        "apply_f64_ms": t_app, "apply_f64_GBps": APPLY_BYTES_F64 * ncell / (t_app * 1e-3) / 1e9,
        "half_sweep_f32_ms": t_rel}
    del ps, x32, b32, r32, x64, y64
    torch.cuda.empty_cache()
    return out


# The paper's 2D iteration counts (Section 5.2): FGMRES(5) preconditioner
# cycles to 1e-6 with W(1,1) on the shifted operator, per grid and column
# (beta, G_s, levels, alpha); counts for the homogeneous model (lambda = 20,
# mu = rho = 1) and for the linear model (rho 2..3, lambda 4..20, mu 1..15).
PAPER_COLUMNS = [(1.0, 10, 2, 0.1), (1.0, 10, 3, 0.4), (1.0, 10, 4, 0.5),
                 (2 / 3, 10, 2, 0.1), (2 / 3, 10, 3, 0.3), (2 / 3, 10, 4, 0.4),
                 (2 / 3, 8, 2, 0.1), (2 / 3, 8, 3, 0.5), (2 / 3, 8, 4, 0.5)]
PAPER_COLUMNS_LINEAR = [(1.0, 10, 2, 0.1), (1.0, 10, 3, 0.4), (1.0, 10, 4, 0.5),
                        (2 / 3, 10, 2, 0.1), (2 / 3, 10, 3, 0.3), (2 / 3, 10, 4, 0.4),
                        (2 / 3, 8, 2, 0.1), (2 / 3, 8, 3, 0.4), (2 / 3, 8, 4, 0.5)]
PAPER_COUNTS = {
    "homogeneous": {(128, 512): [39, 131, 160, 22, 86, 143, 27, 144, 171],
                    (256, 1024): [56, 199, 243, 32, 135, 222, 39, 231, 269],
                    (512, 2048): [79, 256, 332, 40, 144, 275, 50, 294, 294]},
    "linear": {(128, 512): [39, 134, 169, 24, 77, 133, 31, 134, 181],
               (256, 1024): [59, 265, 333, 34, 134, 260, 40, 219, 337],
               (512, 2048): [80, 396, 452, 42, 153, 379, 52, 266, 479]},
}


def paper_tables(args):
    """Readings: h = 1 (grid units); absorbing layer of 20 cells on every
    side; one u_2 point source in the middle of the top row; the coarsest
    solve (LU in the paper) replaced by Vanka-preconditioned GMRES to a 1e-8
    residual drop; float64 cycle.  Only the 3- and 4-level columns on the
    two smaller grids: with 2 levels the coarsest grid is a 5-points-per-
    wavelength Helmholtz problem at shift 0.1, which the iterative stand-in
    for LU does not solve."""
    import numpy as np
    import torch
    from paper_2307_03242_amd import Problem
    from synthetic import constant_media, linear_media, omega_for_ppw
    out = {}
    for model in ("homogeneous", "linear"):
        cols = PAPER_COLUMNS if model == "homogeneous" else PAPER_COLUMNS_LINEAR
        rows = {}
        for shape, printed in PAPER_COUNTS[model].items():
            if shape[1] > 1024:
                continue
            if model == "homogeneous":
                m = constant_media(shape, 20.0, 1.0, 1.0)
            else:
                m = linear_media(shape, (4.0, 20.0), (1.0, 15.0), (2.0, 3.0))
            vs_min = float(np.sqrt(m["mu"] / m["rho"]).min())
            med = [torch.from_numpy(m[k]) for k in ("lam", "mu", "rho")]
            q = torch.zeros((1, 3) + shape, dtype=torch.complex128)
            q[0, 1, 1, shape[1] // 2] = 1.0
            q = q.cuda()
            got = []
            for (beta, gs, levels, alpha) in cols:
                if levels == 2:
                    got.append(None)
                    continue
                prob = Problem(*med, h=1.0, omega=omega_for_ppw(vs_min, 1.0, gs), gamma=0.01, alpha=alpha,
                               beta=beta, abl_width=20.0, abl_amp=2.0, levels=levels, nu1=1, nu2=1, cycle="W",
                               damping=(0.55, 0.35, 0.25), coarse_mode="krylov", coarse_sweeps=2,
                               coarse_restart=10, coarse_maxit=400, coarse_rtol=1e-8,
                               precond_dtype=torch.complex128)
                _, info, code = prob.solve(q, rtol=1e-6, maxit=600)
                got.append(info[0]["iters"] if code == 0 else None)
                prob.close()
                print("%s %dx%d beta=%.3f Gs=%d levels=%d alpha=%.2f: %s (paper %d)"
                      % (model, shape[1], shape[0], beta, gs, levels, alpha, got[-1], printed[len(got) - 1]),
                      file=sys.stderr, flush=True)
            rows["%dx%d" % (shape[1], shape[0])] = {"ours": got, "paper": printed,
                                                    "ratio": [None if g is None else round(g / p, 3)
                                                              for g, p in zip(got, printed)]}
        out[model] = {"columns": [{"beta": round(b, 4), "G_s": g, "levels": l, "alpha": a} for b, g, l, a in cols],
                      "rows": rows}
    return out


# The paper's 3D counts (Section 5.3, Overthrust model): preconditioner
# cycles to 1e-6, K-cycles; columns (beta, G_s, levels, alpha); the model's
# grid shapes (x_1 x x_2 x depth).
PAPER_3D_COLUMNS = [(1.0, 10, 3, 0.4), (1.0, 10, 4, 0.5), (2 / 3, 10, 3, 0.3), (2 / 3, 10, 4, 0.4),
                    (2 / 3, 8, 3, 0.4), (2 / 3, 8, 4, 0.5)]
PAPER_3D_COUNTS = {(128, 128, 56): [39, 72, 28, 31, 30, 44],
                   (256, 256, 96): [77, 175, 49, 51, 54, 70],
                   (384, 384, 136): [121, None, 63, 73, 67, 114]}  # None: printed as > 200


def paper_3d(args):
    """The Overthrust model is not available: the seeded layered + Gaussian
    media of the benchmark (seed 3) on the same grid shapes stand in, with
    the benchmark's absorbing layer (16 cells), centred u_3 source and
    damping; float32 K(1,1) cycle in float64 FGMRES(5).  The coarsest solve
    follows the paper's stopping rule (a residual drop of 0.1, at most 25
    inner FGMRES(5) steps), preconditioned by one Vanka sweep."""
    import torch
    from paper_2307_03242_amd import Problem
    from synthetic import make_media, point_source, omega_for_ppw
    rows = {}
    for (n1, n2, n3), printed in PAPER_3D_COUNTS.items():
        shape = (n3, n2, n1)
        m = make_media(shape, args.seed)
        med = [torch.from_numpy(m[k]).cuda() for k in ("lam", "mu", "rho")]
        q = torch.from_numpy(point_source(shape)[None]).cuda()
        got = []
        for (beta, gs, levels, alpha) in PAPER_3D_COLUMNS:
            cfg = solver_cfg(args, omega_for_ppw(m["vs"].min(), 1.0, gs), levels=levels)
            cfg.update(alpha=alpha, beta=beta, coarse_mode="krylov", coarse_sweeps=1, coarse_maxit=25,
                       coarse_rtol=0.1)
            prob = Problem(*med, precond_dtype=torch.complex64, **cfg)
            _, info, code = prob.solve(q, rtol=args.rtol, maxit=400)
            got.append(info[0]["iters"] if code == 0 else None)
            prob.close()
            print("3D %dx%dx%d beta=%.3f Gs=%d levels=%d alpha=%.2f: %s (paper %s)"
                  % (n1, n2, n3, beta, gs, levels, alpha, got[-1], printed[len(got) - 1]), file=sys.stderr, flush=True)
        rows["%dx%dx%d" % (n1, n2, n3)] = {"ours": got, "paper": printed}
        del med
        torch.cuda.empty_cache()
    return {"columns": [{"beta": round(b, 4), "G_s": g, "levels": l, "alpha": a} for b, g, l, a in PAPER_3D_COLUMNS],
            "rows": rows}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(each source/problem would shard independently across GPUs).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2307_03242_amd import Problem
    from synthetic import make_media, point_source, omega_for_ppw

    torch.cuda.set_device(0)
    if args.paper_tables:
        print(json.dumps({"paper_tables": paper_tables(args)}), flush=True)
        return
    if args.paper_3d:
        print(json.dumps({"paper_3d": paper_3d(args)}), flush=True)
        return
    n = args.n
    shape = (n, n, n)
    m = make_media(shape, args.seed)
    h = 1.0
    omega = omega_for_ppw(m["vs"].min(), h, 10)
    damping = [float(v) for v in args.damping.split(",")]
    cfg = dict(h=h, omega=omega, gamma=0.01, alpha=args.alpha, beta=2 / 3, abl_width=args.abl * h,
               abl_amp=2.0, levels=args.levels, nu1=1, nu2=1, cycle=args.cycle, damping=damping, coarse_mode=args.coarse,
               coarse_sweeps=args.coarse_sweeps, coarse_restart=5, coarse_maxit=args.coarse_maxit,
               coarse_rtol=args.coarse_rtol)
    lam = torch.from_numpy(m["lam"]).cuda()
    mu = torch.from_numpy(m["mu"]).cuda()
    rho = torch.from_numpy(m["rho"]).cuda()
    q = torch.from_numpy(point_source(shape)[None]).cuda()
    stream = torch.cuda.current_stream()
    if args.pmc_target:
        from synthetic import random_field
        src = torch.ones(1 << 27, dtype=torch.complex64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        pr = Problem(lam, mu, rho, precond_dtype=torch.complex64, **cfg)
        xx = torch.from_numpy(random_field(shape, 1)).cuda().to(torch.complex64)
        bb = torch.from_numpy(random_field(shape, 2)).cuda().to(torch.complex64)
        rr = torch.empty_like(xx)
        yy = torch.empty_like(xx)
        for _ in range(4):
            pr.residual(bb, xx, shifted=True, out=rr)
        for _ in range(4):
            pr.apply(xx, out=yy)
        for _ in range(4):
            pr.relax(bb, yy, 1)
        for _ in range(4):
            pr.restrict_residual(bb, xx)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_target": True, "copy_bytes_each_way": 1 << 30, "n": n,
                          "resid_algorithmic_bytes": RESID_BYTES_F32 * n ** 3}), flush=True)
        return

    def timed_solves(prob):
        u = torch.empty_like(q)
        infos = []
        for _ in range(args.warmup):
            prob.solve(q, rtol=args.rtol, maxit=args.maxit, out=u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, info, code = prob.solve(q, rtol=args.rtol, maxit=args.maxit, out=u)
            infos.append(info[0])
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, infos, u

    def split(info):
        # GPU time of one solve by phase (HIP events on the library's stream):
        # preconditioner cycles, outer operator, Gram-Schmidt with its reductions
        # and host round trips; wall = the call's wall clock
        return {"precond": info["t_precond_ms"], "outer_apply": info["t_apply_ms"],
                "orthogonalisation": info["t_orth_ms"], "wall": info["t_total_ms"]}

    p64 = Problem(lam, mu, rho, precond_dtype=torch.complex128, **cfg)
    t64, info64, u64 = timed_solves(p64)
    u64 = u64.clone()
    del p64
    torch.cuda.empty_cache()
    p32 = Problem(lam, mu, rho, precond_dtype=torch.complex64, **cfg)
    t32, info32, u32 = timed_solves(p32)
    rel_diff = float(torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64))

    # stencil bandwidth, HIP events on the stream the library uses: the
    # operator apply in both precisions, and the float32 residual on the
    # shifted operator (the dominant kernel of the float32-cycle solve)
    from synthetic import random_field
    x = torch.from_numpy(random_field(shape, 1)).cuda()
    apply = {}
    for name, dt, nbytes in (("f64", torch.complex128, APPLY_BYTES_F64), ("f32", torch.complex64, APPLY_BYTES_F32)):
        xx = x.to(dt)
        yy = torch.empty_like(xx)
        p32.apply(xx, out=yy)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.apply_reps):
            p32.apply(xx, out=yy)
        ev1.record(stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1) / args.apply_reps
        apply[name] = dict(ms=ms, gbs=nbytes * n ** 3 / (ms * 1e-3) / 1e9)
    xx = x.to(torch.complex64)
    bb = torch.from_numpy(random_field(shape, 2)).cuda().to(torch.complex64)
    rr = torch.empty_like(xx)
    p32.residual(bb, xx, shifted=True, out=rr)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.apply_reps):
        p32.residual(bb, xx, shifted=True, out=rr)
    ev1.record(stream)
    ev1.synchronize()
    resid_ms = ev0.elapsed_time(ev1) / args.apply_reps
    resid_gbs = RESID_BYTES_F32 * n ** 3 / (resid_ms * 1e-3) / 1e9
    del x, xx, bb, rr

    # the plain V-cycle: 4-level V(1,1), float32 against
    # float64 (a short untimed solve that tunes and records the graphs, then
    # one timed solve with up to 1500 iterations)
    vcyc = {}
    if not args.no_extras and args.cycle != "V":
        cfgv = dict(cfg, cycle="V")
        for name, dt in (("fp64", torch.complex128), ("fp32_precond", torch.complex64)):
            pv = Problem(lam, mu, rho, precond_dtype=dt, **cfgv)
            pv.solve(q, rtol=args.rtol, maxit=10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, iv, cv = pv.solve(q, rtol=args.rtol, maxit=1500)
            torch.cuda.synchronize()
            vcyc[name] = {"solves_per_s": 1.0 / (time.perf_counter() - t0), "iters": iv[0]["iters"],
                          "relres": iv[0]["relres"], "code": cv}
            del pv
            torch.cuda.empty_cache()
        vcyc["speedup_fp32_vs_fp64"] = vcyc["fp32_precond"]["solves_per_s"] / vcyc["fp64"]["solves_per_s"]

    value = 1.0 / t32
    it32 = int(np.median([i["iters"] for i in info32]))
    it64 = int(np.median([i["iters"] for i in info64]))
    same_kernel = stencil_source_hash() == RESID_TRAFFIC_SOURCE
    # algorithmic bytes per outer iteration on the finest level (float32
    # cycle, per cell, from the per-unit figures): nu1 = nu2 = 1 red-black
    # sweeps = 4 Vanka passes and 3 residuals (the first half-sweep starts
    # from zero), 1 fused residual restriction, 1 prolongation; outer float64:
    # the float32-input operator and classical Gram-Schmidt (j = 3 average)
    cells = n ** 3
    fine = {"residual_3x": 3 * RESID_BYTES_F32, "vanka_4x": 4 * 104, "restrict_residual": 76 + 4,
            "prolong": 68, "outer_apply_f32in": 32 + 64 + 24, "gram_schmidt_j3": (2 * 3 + 3) * 64 + 64}
    out = {
        "metric": "256^3 solves/s to 1e-6 residual, FP32-precond vs FP64; stencil HBM GB/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 cycle / c128 Krylov",
        "data": "synthetic",
        "config": {
            "workload": "3D %d^3 elastic Helmholtz, layered+Gaussian media seed %d, 10 ppw, gamma 0.01, "
                        "ABL %d, 1 point source; FGMRES(5) to %.0e with %d-level %s(1,1) on the shifted "
                        "operator (alpha %.2f), float32 cycle" % (n, args.seed, args.abl, args.rtol,
                                                                  args.levels, args.cycle, args.alpha),
            "grid": [n, n, n], "levels": args.levels, "cycle": args.cycle, "alpha": args.alpha, "beta": 2 / 3,
            "coarse": "%s(sweeps=%d, maxit=%d)" % (args.coarse, args.coarse_sweeps, args.coarse_maxit),
            "parallelism": "single GPU",
        },
        "fp64": {"solves_per_s": 1.0 / t64, "ms_per_solve": t64 * 1e3, "iters": it64,
                 "relres": info64[-1]["relres"], "split_ms": split(info64[-1]),
                 "kernels_per_iteration": info64[-1]["kernels"] / max(1, info64[-1]["iters"])},
        "fp32_precond": {"solves_per_s": value, "iters": it32, "relres": info32[-1]["relres"],
                         "rel_diff_vs_fp64_solution": rel_diff, "split_ms": split(info32[-1]),
                         "kernels_per_iteration": info32[-1]["kernels"] / max(1, info32[-1]["iters"]),
                         "algorithmic_GB_per_iteration_finest": {k: v * cells / 1e9 for k, v in fine.items()}},
        "vcycle_4level": vcyc,
        "speedup_fp32_vs_fp64": t64 / t32,
        "apply": {"f64_ms": apply["f64"]["ms"], "f64_GBps": apply["f64"]["gbs"],
                  "f32_ms": apply["f32"]["ms"], "f32_GBps": apply["f32"]["gbs"]},
        "roofline": {"bound": "hbm", "achieved": resid_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": resid_gbs / HBM_PEAK_GBS,
                     "traffic": (RESID_TRAFFIC_BYTES / (resid_ms * 1e-3) / 1e9
                                 if RESID_TRAFFIC_BYTES and n == 256 and same_kernel else None),
                     "kernel": "residual b - H_s x, complex64, %d^3 (%d B/cell), %.3f ms per launch"
                               % (n, RESID_BYTES_F32, resid_ms)},
    }
    del p32
    torch.cuda.empty_cache()
    if not args.no_extras:
        try:
            out["production_forms"] = extras(args)
        except Exception as e:  # report, never hide
            out["production_forms"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(args, it32, cfg)
        except Exception as e:  # report, never hide
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
