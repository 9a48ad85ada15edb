"""Benchmark of the libsdme hot path on one MI355X.

Workload (default): compress_p4 -- unit cube of 47^3 hexahedra, P = 4,
Q = 6 Gauss points per direction, SDME-H basis (k = 0.5, lambda = 100),
compressible neo-Hookean E = 1e3, nu = 0.3; z = 0 clamped, z = 1 moved by
(0, 0, -0.2) (20 % compression); 6,751,269 slots, 20,253,807 DOFs.  Initial
guess: the affine 20 % compression plus a seeded U(-a, a) perturbation of
every free coefficient, a = 1e-3 h (h the element edge) (synthetic input; the paper's meshes are not
available).

One step = one Newton-Raphson iteration of the hot path from that fixed
initial state: internal force R(u) with the linearisation state, the Jacobi
diagonal, the Jacobi-PCG solve of K_T du = -R to 1e-8 relative residual in
mixed precision (FP32 inner PCG with FP32 state/operator/vectors and FP64
dots, FP64 defect correction), and the update u += du.  value = tangent
applies x DOFs / step time (GDOF/s, whole step).  Besides the timed steps the
same Newton iteration runs once with FP64 PCG (newton_iteration: mixed vs
FP64) and the load-stepped Newton-PCG solve to 1e-8 runs in both
precisions (newton_pcg), the oracle is timed on a bounded sample of the same workload on
the host with all threads and with one (cpu_baseline), and the dominant kernel (FP32 stored-state tangent
action in the inner PCG) is timed per launch by HIP events on its stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve]
       [--no-cpu-baseline] [--kernel-table]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tangent-apply GDOF/s; Newton-PCG solve to 1e-8, mixed-FP32 vs FP64"
HBM_PEAK_GBS = 8000.0
FP32_PEAK = 157.3   # TFLOP/s (datasheet, dense)
FP64_PEAK = 78.6
# flops of the linearised stress dP = mu dF + c1 (G dF G)^T + lam tr(G dF) G^T
# at one Gauss point, with the 2/h and quadrature-weight scalings
POINTWISE_FLOPS = 174


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROFILE = os.path.join(ROOT, "profiles", "k_tangent_fp32_state__compress_p4.md")
KERNEL_SOURCES = ("paper_2104_13466_amd/csrc/elem_kernels.hip",
                  "paper_2104_13466_amd/csrc/sdme_device.h")


def measured_traffic():
    """HBM bytes per launch of the FP32 stored-state tangent kernel from the
    committed counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or
    None when the element-kernel sources changed since it was taken."""
    import hashlib
    try:
        kv = {}
        for line in open(PROFILE):
            if " = " in line:
                k, v = line.strip().split(" = ", 1)
                kv[k] = v
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if kv.get("kernel_sources_sha256") != h.hexdigest()[:16]:
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def setup(name, kind=None, k=0.5, lambda_h=100.0, ordered=False):
    import torch

    from paper_2104_13466_amd import inputs
    from paper_2104_13466_amd.sdme import Context
    w = dict(inputs.WORKLOADS[name])
    if kind is not None:
        w["kind"] = kind
    n, L, P = w["n"], w["L"], w["P"]
    ctx = Context(n, L, P, basis=w["kind"], k=k, lambda_h=lambda_h, dirichlet=w["dirichlet"],
                  ordered=ordered)
    lam0, mu0 = inputs.lame(w["E"], w["nu"])
    dev = torch.device("cuda")
    mu = torch.full((ctx.E,), mu0, dtype=torch.float64, device=dev)
    lam = torch.full((ctx.E,), lam0, dtype=torch.float64, device=dev)
    mat = Context.material(mu, lam, w["rho"])
    G = np.zeros((3, 3))
    G[2, 2] = -0.2
    free = 1.0 - ctx.dirichlet_flags().astype(np.float64)
    amp = 1e-3 * min(L[i] / n[i] for i in range(3))
    u0 = ctx.affine_field([0, 0, 0], G) + free * inputs.random_coeffs(w["seed"], n, P, amp)
    u0 = torch.tensor(u0, device=dev)
    return w, ctx, mat, u0


def newton_iteration(ctx, mat, prec, u, R, du, rtol):
    """R(u) (masked) -> psi = -R -> PCG (K_T(u) du = psi) -> u += du."""
    from paper_2104_13466_amd.sdme import FP64, MASK_BC
    ctx.internal_force(mat, FP64, u, R, flags=MASK_BC)
    ctx.axpby(-1.0, R, 0.0, R)
    st = ctx.jacobi_pcg(mat, prec, R, du, u_lin=u, rtol=rtol)
    ctx.axpby(1.0, du, 1.0, u)
    return st


def kernel_table(ctx, mat, u0):
    """Per-launch times of the element operators at the workload (HIP events)."""
    import torch

    from paper_2104_13466_amd.sdme import FP32, FP64
    N = 3 * ctx.Nn
    rows = []
    for prec, dt in ((FP64, torch.float64), (FP32, torch.float32)):
        u = u0.to(dt)
        v = torch.rand(N, dtype=dt, device="cuda")
        y = torch.zeros_like(v)
        st = torch.empty(ctx.nqp * 10, dtype=dt, device="cuda")
        ctx.linearize(mat, prec, u, st)
        cases = [
            ("tangent_state", lambda: ctx.tangent_apply(mat, prec, v, y, state=st)),
            ("tangent_recompute", lambda: ctx.tangent_apply(mat, prec, v, y, u_lin=u)),
            ("internal_force", lambda: ctx.internal_force(mat, prec, u, y)),
            ("force_and_state", lambda: ctx.internal_force(mat, prec, u, y, state=st)),
            ("mass", lambda: ctx.mass_apply(1.0, prec, v, y)),
            ("jacobi_diag", lambda: ctx.jacobi_diag(mat, prec, st, 0.0, y)),
        ]
        # An idle GPU runs the first tens of milliseconds of work below its
        # sustained clock: warm up on the first case for ~0.2 s before timing.
        warm_until = time.perf_counter() + 0.2
        while time.perf_counter() < warm_until:
            cases[0][1]()
            torch.cuda.synchronize()
        for name, fn in cases:
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            rows.append(("fp64" if prec == FP64 else "fp32", name, ms, N / ms / 1e6))
            log("kernel %-4s %-18s %8.3f ms/call  %7.2f GDOF/s (incl. output fill)" % rows[-1])
    return rows


def mass_roofline(ctx):
    """The mass action (Kronecker stencil) on the workload mesh: per-launch
    time (HIP events on the stream the library launches on, 50 launches after
    ~0.3 s of warm-up launches) against its algorithmic bytes, v read and y
    written once."""
    import torch

    from paper_2104_13466_amd.sdme import FP32, FP64
    N = 3 * ctx.Nn
    out = {}
    for prec, dt, word in ((FP32, torch.float32, 4), (FP64, torch.float64, 8)):
        v = torch.rand(N, dtype=dt, device="cuda")
        y = torch.zeros_like(v)
        # ~0.3 s of launches first: the GPU comes out of the long solves above
        # at a clock that the short streaming kernel does not see right away
        warm_until = time.perf_counter() + 0.3
        while time.perf_counter() < warm_until:
            for _ in range(10):
                ctx.mass_apply(1.0, prec, v, y)
            torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(50):
            ctx.mass_apply(1.0, prec, v, y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 50
        gbs = 2 * word * N / (ms * 1e-3) / 1e9
        out["k_mass_" + ("fp32" if prec == FP32 else "fp64")] = {
            "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(ms, 4),
            "algorithmic_bytes_per_launch": 2 * word * N}
        log("mass %s %.4f ms %.0f GB/s" % ("fp32" if prec == FP32 else "fp64", ms, gbs))
    return out


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device copy of known size (nbytes read + nbytes written per
    launch): the reference that scales the HBM byte counters of the kernels."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: %d x %d bytes" % (reps, nbytes))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, seconds=10.0, sub_n=24):
    """The oracle's direct tangent action timed on the host on a sub-box of the
    workload mesh (same P, Q, basis, element size), with the OpenMP threads the
    environment gives it."""
    from oracle import basis as ob
    from oracle import fem
    from paper_2104_13466_amd import inputs
    P, Q = w["P"], w["P"] + 2
    n = w["n"]
    sub = (min(sub_n, n[0]), min(sub_n, n[1]), min(sub_n, n[2]))
    h = [w["L"][i] / n[i] for i in range(3)]
    b, x, wq, B, D = ob.build(P, Q, w["kind"])
    mesh = fem.Mesh(sub[0], sub[1], sub[2], P, Q, h, B, D, wq)
    lam0, mu0 = inputs.lame(w["E"], w["nu"])
    mu = np.full(mesh.E, mu0)
    lam = np.full(mesh.E, lam0)
    u = inputs.random_coeffs(w["seed"], sub, P, 1e-3)
    v = inputs.uniform(w["seed"], u.size, -1, 1, stream=3)
    t0 = time.perf_counter()
    k = 0
    while True:
        mesh.tangent_apply(mu, lam, u, v)
        k += 1
        if time.perf_counter() - t0 >= seconds:
            break
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": k * 3 * mesh.Nn / t / 1e9, "unit": "GDOF/s", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": "%d x tangent action on a %dx%dx%d-element sub-box (P=%d, %d DOF) of the "
                      "workload mesh, %.1f s" % (k, sub[0], sub[1], sub[2], P, 3 * mesh.Nn, t)}


def cpu_baseline_single(workload):
    """The same measurement with one OpenMP thread, in a child process (the
    oracle's thread count is fixed when its library loads)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--workload", workload,
                        "--cpu-baseline-only", "--cpu-sub", "10"],
                       env=env, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        log("single-thread cpu baseline failed: %s" % r.stderr[-500:])
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def full_solve(ctx, mat, u0, a):
    """Newton-PCG time-to-solution in FP64 and mixed: the top displacement
    (a.solve_compression of the height) is applied in equal increments (load
    stepping); each increment starts from the previous solution plus the
    affine increment and runs the damped Newton of sdme_newton_static to 1e-8
    with PCG to 1e-8."""
    import torch

    from paper_2104_13466_amd.sdme import FP32, FP64
    G = np.zeros((3, 3))
    G[2, 2] = -a.solve_compression / a.increments
    inc = torch.tensor(ctx.affine_field([0, 0, 0], G), device="cuda")
    out = {}
    sols = {}
    for prec, name in ((FP64, "fp64"), (FP32, "mixed")):
        u = torch.zeros_like(u0)
        tot = {"newton": 0, "pcg_iterations": 0, "outer": 0}
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for k in range(a.increments):
            ctx.axpby(1.0, inc, 1.0, u)
            st = ctx.newton_static(mat, prec, u, newton_rtol=a.rtol, pcg_rtol=a.rtol)
            for key in tot:
                tot[key] += st["iterations" if key == "pcg_iterations" else key]
            log("solve %s increment %d: %s" % (name, k, st))
        torch.cuda.synchronize()
        tot["seconds"] = round(time.perf_counter() - ts, 3)
        out[name] = tot
        sols[name] = u
    out["speedup_mixed_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 3)
    out["max_rel_diff_mixed_vs_fp64"] = ((sols["mixed"] - sols["fp64"]).abs().max() /
                                         sols["fp64"].abs().max()).item()
    out["increments"] = a.increments
    out["compression_reached"] = a.solve_compression
    out["compression_configured"] = 0.2
    out["note"] = ("load-stepped to %.0f %% nominal compression: at 47^3, P = 4 the tangent "
                   "stops being positive definite near the clamped edges beyond about 16 %%"
                   % (100 * a.solve_compression))
    return out


# ------------------------------------------------------------------ cases
# Further measurements of the hot path on the other workloads; each prints one
# JSON line of its own (python bench.py --case NAME).
KIND_NAMES = {0: "nodal", 1: "modal", 2: "sdme_m", 3: "sdme_k", 4: "sdme_h"}


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, 1e3 * (time.perf_counter() - t0)


def case_sweep(a):
    """Polynomial-order sweep at ~2e7 DOF (P = 2, 4, 6, 8, SDME-H): operator
    launch times and one Newton iteration (PCG to 1e-8) in FP64 and mixed;
    then the same mixed Newton iteration at P = 4 for every basis kind."""
    import gc

    import torch

    from paper_2104_13466_amd.sdme import FP32, FP64
    rows = []
    for wl in ("compress_p2", "compress_p4", "compress_p6", "compress_p8"):
        w, ctx, mat, u0 = setup(wl)
        N = 3 * ctx.Nn
        row = {"workload": wl, "P": w["P"], "dofs": N, "elements": ctx.E}
        row["kernel_ms"] = {"%s_%s" % (r[0], r[1]): round(r[2], 4) for r in kernel_table(ctx, mat, u0)}
        R = torch.zeros(N, dtype=torch.float64, device="cuda")
        du = torch.zeros_like(R)
        for prec, name in ((FP64, "fp64"), (FP32, "mixed")):
            u = u0.clone()
            st, ms = timed(lambda: newton_iteration(ctx, mat, prec, u, R, du, a.rtol))
            row[name] = {"ms": round(ms, 1), "pcg_iterations": st["iterations"],
                         "replacements": st["outer"], "rel_residual": st["rel_residual"]}
            log("%s %s: %s" % (wl, name, row[name]))
        row["speedup_mixed_vs_fp64"] = round(row["fp64"]["ms"] / row["mixed"]["ms"], 3)
        rows.append(row)
        del ctx, mat, u0, R, du, u
        gc.collect()
        torch.cuda.empty_cache()
    bases = []
    for kind in (4, 2, 3, 1, 0):
        w, ctx, mat, u0 = setup("compress_p4", kind=kind)
        N = 3 * ctx.Nn
        R = torch.zeros(N, dtype=torch.float64, device="cuda")
        du = torch.zeros_like(R)
        u = u0.clone()
        from paper_2104_13466_amd.sdme import MASK_BC

        def one():
            ctx.internal_force(mat, FP64, u, R, flags=MASK_BC)
            ctx.axpby(-1.0, R, 0.0, R)
            return ctx.jacobi_pcg(mat, FP32, R, du, u_lin=u, rtol=a.rtol, maxit=30000, check=False)
        st, ms = timed(one)
        bases.append({"basis": KIND_NAMES[kind], "pcg_iterations": st["iterations"],
                      "status": st["status"], "ms": round(ms, 1),
                      "rel_residual": st["rel_residual"]})
        log("basis %s: %s" % (KIND_NAMES[kind], bases[-1]))
        del ctx, mat, u0, R, du, u
        gc.collect()
        torch.cuda.empty_cache()
    return {"case": "sweep", "rtol": a.rtol, "rows": rows, "bases_p4_mixed_newton_iteration": bases}


def case_newmark(a):
    """Implicit Newmark (beta = 1/4, gamma = 1/2) on the 16x4x4 cantilever, P = 4:
    dead tip traction -z on x = 4 ramped linearly to 5.0 over 20 steps of
    dt = 0.1, Newton to 1e-8 with Jacobi-PCG to 1e-8; SDME-H, SDME-M and the
    Lagrange-nodal basis, FP64 and mixed."""
    import torch

    from paper_2104_13466_amd import inputs
    from paper_2104_13466_amd.sdme import FP32, FP64
    w = inputs.WORKLOADS["cantilever_p4"]
    runs = []
    for kind in (4, 2, 0):
        runs.extend(newmark_runs(w, kind, 0.5, 100.0, (FP64, FP32)))
    return {"case": "newmark", "workload": "cantilever_p4: 16x4x4 hexahedra on 4x1x1, P=4, "
            "clamped x=0, tip traction ramped to 5.0 over 20 steps, dt=0.1",
            "dofs": 3 * inputs.num_nodes(w["n"], w["P"]), "runs": runs}


def newmark_runs(w, kind, k, lambda_h, precs):
    """20 Newmark steps of the cantilever workload with one basis, per precision."""
    import torch

    from paper_2104_13466_amd import inputs
    from paper_2104_13466_amd.sdme import FP64, Context
    runs = []
    lam0, mu0 = inputs.lame(w["E"], w["nu"])
    ctx = Context(w["n"], w["L"], w["P"], basis=kind, k=k, lambda_h=lambda_h,
                  dirichlet=w["dirichlet"])
    mat = Context.material(torch.full((ctx.E,), mu0, dtype=torch.float64, device="cuda"),
                           torch.full((ctx.E,), lam0, dtype=torch.float64, device="cuda"),
                           w["rho"])
    N = 3 * ctx.Nn
    funit = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.face_traction(1, [0.0, 0.0, -1.0], funit)
    sols = {}
    for prec, name in [(q, "fp64" if q == FP64 else "mixed") for q in precs]:
        u = torch.zeros(N, dtype=torch.float64, device="cuda")
        v = torch.zeros_like(u)
        acc = torch.zeros_like(u)
        f = torch.zeros_like(u)
        tot = {"newton": 0, "pcg_iterations": 0, "replacements": 0}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for step in range(1, 21):
            f.copy_(funit * (5.0 * step / 20))
            st = ctx.newmark_newton_step(mat, prec, u, v, acc, f, 0.1)
            tot["newton"] += st["newton"]
            tot["pcg_iterations"] += st["iterations"]
            tot["replacements"] += st["outer"]
        torch.cuda.synchronize()
        tot["seconds"] = round(time.perf_counter() - t0, 3)
        # tip deflection: z-displacement of the slot at (x = 4, y = 0.5, z = 0.5)
        Nx, Ny = w["n"][0] * w["P"] + 1, w["n"][1] * w["P"] + 1
        Nz = w["n"][2] * w["P"] + 1
        g = ((Nz // 2) * Ny + Ny // 2) * Nx + Nx - 1
        tot["tip_uz"] = u[2 * ctx.Nn + g].item()
        sols[name] = u
        runs.append(dict(basis=KIND_NAMES[kind], k=k, lambda_h=lambda_h, precision=name,
                         **tot))
        log("newmark %s %s: %s" % (KIND_NAMES[kind], name, runs[-1]))
    if "mixed" in sols and "fp64" in sols:
        runs[-1]["max_rel_diff_vs_fp64"] = ((sols["mixed"] - sols["fp64"]).abs().max() /
                                            sols["fp64"].abs().max()).item()
    del ctx
    return runs


def case_params(a):
    """Basis parameters the paper varies: the SDME-H lambda tied to the Newmark
    shift (lambda = b1 = 4 / dt^2 = 400 for dt = 0.1) against the default 100
    on the cantilever, and the SD exponent k = 0, 0.5, 1 on one mixed Newton
    iteration of the P = 4 compression."""
    import gc

    import torch

    from paper_2104_13466_amd import inputs
    from paper_2104_13466_amd.sdme import FP32, FP64, MASK_BC
    w = inputs.WORKLOADS["cantilever_p4"]
    newmark = []
    for lam_h in (100.0, 400.0):
        newmark.extend(newmark_runs(w, 4, 0.5, lam_h, (FP64,)))
    static = []
    for kind, k in ((4, 0.0), (4, 0.5), (4, 1.0), (3, 0.0), (3, 1.0), (2, 0.5)):
        w2, ctx, mat, u0 = setup("compress_p4", kind=kind, k=k)
        N = 3 * ctx.Nn
        R = torch.zeros(N, dtype=torch.float64, device="cuda")
        du = torch.zeros_like(R)

        def one():
            ctx.internal_force(mat, FP64, u0, R, flags=MASK_BC)
            ctx.axpby(-1.0, R, 0.0, R)
            return ctx.jacobi_pcg(mat, FP32, R, du, u_lin=u0, rtol=a.rtol, maxit=30000, check=False)
        st, ms = timed(one)
        static.append({"basis": KIND_NAMES[kind], "k": k, "pcg_iterations": st["iterations"],
                       "status": st["status"], "ms": round(ms, 1)})
        log("params %s" % static[-1])
        del ctx, mat, u0, R, du
        gc.collect()
        torch.cuda.empty_cache()
    return {"case": "params", "newmark_cantilever_p4_fp64": newmark,
            "compress_p4_mixed_newton_iteration": static}


def case_explicit(a):
    """Central-difference impact on the 64x64x16 block (4x4x1, P = 3, SDME-M):
    v0 = -0.05 c_L z onto the rigid plane z = 0 (penalty 10E/h), dt from the
    power iteration at CFL 0.5, FP32 internal force, FP64 update and mass
    solve; a.steps_explicit steps with the energy balance checked in FP64."""
    import torch

    from paper_2104_13466_amd import inputs
    from paper_2104_13466_amd.sdme import FP32, FP64, Context
    w = inputs.WORKLOADS["impact_p3"]
    lam0, mu0 = inputs.lame(w["E"], w["nu"])
    ctx = Context(w["n"], w["L"], w["P"], basis=w["kind"], dirichlet=w["dirichlet"])
    mat = Context.material(torch.full((ctx.E,), mu0, dtype=torch.float64, device="cuda"),
                           torch.full((ctx.E,), lam0, dtype=torch.float64, device="cuda"), w["rho"])
    N = 3 * ctx.Nn
    h = w["L"][2] / w["n"][2]
    eps = 10 * w["E"] / h
    cont = (eps, 0.0)
    cL = np.sqrt(w["E"] * (1 - w["nu"]) / (w["rho"] * (1 + w["nu"]) * (1 - 2 * w["nu"])))
    v0 = torch.tensor(ctx.affine_field([0, 0, -0.05 * cL], np.zeros((3, 3))), device="cuda")
    x0 = torch.tensor(inputs.uniform(w["seed"], N, -1, 1, stream=5), device="cuda")
    zero = torch.zeros(N, dtype=torch.float64, device="cuda")
    lmax, ms_l = timed(lambda: ctx.lambda_max(mat, zero, x0, iters=60, contact=cont, mass_rtol=1e-8))
    dt = 0.5 * 2.0 / np.sqrt(lmax)
    steps = a.steps_explicit
    # start step u_1 = u_0 + dt v0 + dt^2/2 a_0 from u_0 = 0
    u_prev = torch.zeros(N, dtype=torch.float64, device="cuda")
    u_cur = torch.zeros_like(u_prev)
    u_next = torch.zeros_like(u_prev)
    ctx.explicit_step(mat, FP32, None, u_prev, u_cur, dt, v0=v0, contact=cont, mass_rtol=1e-8)
    energies = []
    mass_its = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, steps):
        st = ctx.explicit_step(mat, FP32, u_prev, u_cur, u_next, dt, contact=cont, mass_rtol=1e-8)
        mass_its += st["mass_iterations"]
        if k % max(1, steps // 10) == 0 or k == steps - 1:
            ke, se, ce = ctx.energies(mat, u_prev, u_cur, u_next, dt, contact=cont)
            energies.append({"step": k, "kinetic": ke, "strain": se, "contact": ce,
                             "total": ke + se + ce})
        u_prev, u_cur, u_next = u_cur, u_next, u_prev
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    e0 = 0.5 * w["rho"] * (0.05 * cL) ** 2 * w["L"][0] * w["L"][1] * w["L"][2]
    drift = max(abs(e["total"] - e0) for e in energies) / e0
    return {"case": "explicit", "workload": "impact_p3: 64x64x16 hexahedra on 4x4x1, P=3, SDME-M, "
            "v0=-0.05 c_L onto a rigid plane, penalty 10E/h, CFL 0.5", "dofs": N,
            "lambda_max": lmax, "dt": dt, "lambda_max_ms": round(ms_l, 1), "steps": steps,
            "seconds": round(sec, 3), "ms_per_step": round(1e3 * sec / max(steps - 1, 1), 3),
            "mass_pcg_iterations_per_step": mass_its / max(steps - 1, 1),
            "initial_kinetic_energy": e0, "max_rel_energy_deviation": drift,
            "energies": energies}


def case_adjoint(a):
    """Differentiable explicit run on the 16^3 cube, P = 4, SDME-M: per-element
    log-normal mu, lam (sigma 0.2), 50 central-difference steps at CFL 0.5,
    J = 1/2 ||u_K - u*||^2 with u* the rollout of the homogeneous material;
    forward (checkpoint every 10 steps) and adjoint backward timed; the gradient
    checked against a central difference (h = 1e-6 relative) along a seeded
    direction."""
    import torch

    from paper_2104_13466_amd import inputs
    from paper_2104_13466_amd.adjoint import RolloutSpec, SdmeExplicitRollout, rollout
    from paper_2104_13466_amd.sdme import Context
    w = inputs.WORKLOADS["adjoint_p4"]
    ctx = Context(w["n"], w["L"], w["P"], basis=w["kind"], dirichlet=w["dirichlet"])
    N = 3 * ctx.Nn
    lam0, mu0 = inputs.lame(w["E"], w["nu"])
    mu, lam = inputs.lognormal_lame(w["seed"], ctx.E, w["E"], w["nu"])
    dev = "cuda"
    mu_t = torch.tensor(mu, device=dev).requires_grad_(True)
    lam_t = torch.tensor(lam, device=dev).requires_grad_(True)
    free = 1.0 - ctx.dirichlet_flags().astype(np.float64)
    cL = np.sqrt(w["E"] * (1 - w["nu"]) / (w["rho"] * (1 + w["nu"]) * (1 - 2 * w["nu"])))
    v0 = torch.tensor(free * inputs.uniform(w["seed"], N, -0.01 * cL, 0.01 * cL, stream=6),
                      device=dev)
    u0 = torch.zeros(N, dtype=torch.float64, device=dev)
    x0 = torch.tensor(inputs.uniform(w["seed"], N, -1, 1, stream=5), device=dev)
    mat = Context.material(mu_t.detach(), lam_t.detach(), w["rho"])
    lmax = ctx.lambda_max(mat, u0, x0, iters=60, mass_rtol=1e-8)
    dt = 0.5 * 2.0 / np.sqrt(lmax)
    steps = 50
    spec0 = RolloutSpec(ctx, w["rho"], u0, v0, dt, steps, torch.zeros_like(u0), checkpoint=10)
    _, target, _, _ = rollout(spec0, torch.full((ctx.E,), mu0, dtype=torch.float64, device=dev),
                              torch.full((ctx.E,), lam0, dtype=torch.float64, device=dev),
                              keep=False)
    target = target.clone()
    spec = RolloutSpec(ctx, w["rho"], u0, v0, dt, steps, target, checkpoint=10)
    J, ms_f = timed(lambda: SdmeExplicitRollout.apply(mu_t, lam_t, spec))
    _, ms_b = timed(lambda: J.backward())
    # central difference along a seeded direction (relative perturbation)
    d_mu = torch.tensor(inputs.uniform(w["seed"], ctx.E, -1, 1, stream=30), device=dev) * mu_t.detach()
    d_lam = torch.tensor(inputs.uniform(w["seed"], ctx.E, -1, 1, stream=31), device=dev) * lam_t.detach()
    h = 1e-6
    with torch.no_grad():
        Jp = rollout(spec, mu_t + h * d_mu, lam_t + h * d_lam, keep=False)[0]
        Jm = rollout(spec, mu_t - h * d_mu, lam_t - h * d_lam, keep=False)[0]
    fd = (Jp - Jm) / (2 * h)
    ad = float((mu_t.grad * d_mu).sum() + (lam_t.grad * d_lam).sum())
    return {"case": "adjoint", "workload": "adjoint_p4: 16^3 hexahedra, P=4, SDME-M, log-normal "
            "mu, lam (sigma 0.2), 50 steps, checkpoint 10", "dofs": N, "dt": dt,
            "J": J.item(), "forward_ms": round(ms_f, 1), "backward_ms": round(ms_b, 1),
            "directional_derivative_adjoint": ad, "directional_derivative_fd": fd,
            "rel_diff": abs(ad - fd) / abs(fd)}


def _golden(name):
    rows = {}
    for line in open(os.path.join(ROOT, "tests", "golden", name)):
        if line.strip() and not line.startswith("#"):
            v = line.split()
            rows[int(v[0])] = [float(x) for x in v[1:]]
    return rows


def case_static(a):
    """Static large-strain fabricated solution of Section 5.1 (u_x = 1.9 sin x
    - x on the 2x2x2 unit cube, x = 0 clamped, tractions of the exact field on
    the other faces, body force -Div P): Newton from u = 0 to 1e-8 with
    Jacobi-PCG to 1e-8, P = 2, 4, 6, 8, for the modal (ST), SDME-M and SDME-H
    bases in FP64 and SDME-H mixed; L2 errors, Newton and PCG iterations and
    time per Newton iteration beside the paper's printed values (Tables
    Tab:Static_error, Tab:NH_average_IT_CGD, Tab:NH_average_Time_CGD)."""
    import torch

    from paper_2104_13466_amd import fabricated as pf
    from paper_2104_13466_amd.sdme import FP32, FP64, Context
    l2 = _golden("static_l2_errors.txt")
    its = _golden("static_cgd_iterations.txt")
    rows = []
    for P in (2, 4, 6, 8):
        for kind, prec in ((1, FP64), (2, FP64), (4, FP64), (4, FP32)):
            ctx = Context((2, 2, 2), (1.0, 1.0, 1.0), P, basis=kind, dirichlet=pf.DIRICHLET_X0)
            lam, mu = pf.lame()
            mat = Context.material(torch.full((ctx.E,), mu, dtype=torch.float64, device="cuda"),
                                   torch.full((ctx.E,), lam, dtype=torch.float64, device="cuda"),
                                   1.0)
            f = torch.zeros(3 * ctx.Nn, dtype=torch.float64, device="cuda")
            pf.static_loads(ctx, f)
            g = pf.static_exact_at_gauss_points(ctx)
            u = torch.zeros_like(f)
            ctx.newton_static(mat, prec, u.clone(), f_ext=f)  # warm-up
            st, ms = timed(lambda: ctx.newton_static(mat, prec, u, f_ext=f, newton_rtol=1e-8,
                                                     pcg_rtol=1e-8, max_pcg=20000))
            err = ctx.l2_error(u, g)
            col = {1: 0, 2: 1, 4: 2}[kind]
            row = {"P": P, "basis": KIND_NAMES[kind], "prec": "fp64" if prec == FP64 else "mixed",
                   "dofs_free": int(l2[P][0]), "l2_error": [float("%.4g" % e) for e in err],
                   "paper_l2_error": l2[P][1:], "newton": st["newton"],
                   "pcg_per_newton": round(st["iterations"] / max(st["newton"], 1), 1),
                   "paper_cgd_per_newton": its[P][1 + col],
                   "ms_per_newton": round(ms / max(st["newton"], 1), 3),
                   "paper_cgd_s_per_newton": its[P][4 + col]}
            log("static %s" % row)
            rows.append(row)
            ctx.close()
    return {"case": "static", "rows": rows}


def case_wave(a):
    """Transient fabricated solution of Section 5.2 (u_x = sin(pi x / 2)
    sin(2 pi t) on the 2x2x2 unit cube to t = 0.25, x = 0 clamped):
    central differences (800 steps; also with the nodal basis and the lumped
    GLL-rule mass) and Newmark (dt = 2e-3, 125 steps, Newton and Jacobi-PCG to
    1e-8), P = 2, 4, 6; L2 errors, iterations and times beside the paper's
    tables (Tab:Transient_NH_L2errorHexa_ST, _SDME_M, _Lagrange,
    Tab:TransientNmk_NH_L2errorHexa_SDME_H, Tab:TransientNmk_NH_NIT_Hexa,
    Tab:TransientNmk_NH_time_Hexa)."""
    import torch

    from paper_2104_13466_amd import fabricated as pf
    from paper_2104_13466_amd.sdme import FP32, FP64, Context
    ref = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "wave_l2_errors.txt")):
        if line.strip() and not line.startswith("#"):
            v = line.split()
            ref[(v[0], v[1], int(v[2]))] = [float(x) for x in v[4:]]
    nit = _golden("wave_newmark_cgd_iterations.txt")

    def mk(P, kind, lumped=False):
        ctx = Context((2, 2, 2), (1.0, 1.0, 1.0), P, basis=kind, dirichlet=pf.DIRICHLET_X0,
                      lumped_mass=lumped)
        lam, mu = pf.lame()
        mat = Context.material(torch.full((ctx.E,), mu, dtype=torch.float64, device="cuda"),
                               torch.full((ctx.E,), lam, dtype=torch.float64, device="cuda"), pf.RHO)
        return ctx, mat

    rows = []
    for P in (2, 4, 6):
        runs = [("explicit", 2, FP64), ("explicit", 2, FP32), ("explicit-lumped", 0, FP64),
                ("newmark", 4, FP64), ("newmark", 4, FP32), ("newmark", 2, FP64),
                ("newmark", 1, FP64)]
        if P <= 4:
            runs.append(("explicit", 1, FP64))
        for scheme, kind, prec in runs:
            ctx, mat = mk(P, kind, lumped=scheme == "explicit-lumped")
            if scheme.startswith("explicit"):
                (u, its), ms = timed(lambda: pf.wave_explicit(ctx, mat, 0.25 / 800, 800, prec))
                row = {"steps": 800, "mass_pcg_per_step": round(its / 800, 1),
                       "ms_per_step": round(ms / 800, 3), "force_prec": "fp64" if prec == FP64 else "fp32"}
            else:
                (u, newton, pcg), ms = timed(lambda: pf.wave_newmark(ctx, mat, 2e-3, 125, prec))
                col = {1: 0, 2: 1, 4: 2}[kind]
                row = {"steps": 125, "newton": newton, "pcg_per_solve": round(pcg / newton, 2),
                       "paper_cgd_per_solve": nit[P][col], "ms_per_step": round(ms / 125, 3),
                       "prec": "fp64" if prec == FP64 else "mixed"}
            err = ctx.l2_error(u, pf.exact_at_gauss_points(ctx, "wave", 0.25))
            key = ("explicit", "lagrange_diag", P) if scheme == "explicit-lumped" else (
                scheme, KIND_NAMES[kind], P)
            row.update({"scheme": scheme, "P": P, "basis": KIND_NAMES[kind],
                        "l2_error": [float("%.4g" % e) for e in err],
                        "paper_l2_error": ref.get(key)})
            log("wave %s" % row)
            rows.append(row)
            ctx.close()
    return {"case": "wave", "rows": rows}


def case_quartic(a):
    """Newmark runs of the fabricated solution u_x = x^4 sin(2 pi t) of
    Section 5.2 (2x2x2 unit cube, T = 0.025, SDME-H, Newton and PCG to
    1e-10): spatial convergence at dt = 3.9e-4 for P = 2..6 and time
    convergence at P = 5 for 8..128 steps (the paper shows both only in a
    figure, stating exponential convergence in space and a quadratic rate in
    time)."""
    import torch

    from paper_2104_13466_amd import fabricated as pf
    from paper_2104_13466_amd.sdme import FP64, Context
    T = 0.025

    def run(P, nsteps):
        ctx = Context((2, 2, 2), (1.0, 1.0, 1.0), P, basis=4, dirichlet=pf.DIRICHLET_X0)
        lam, mu = pf.lame()
        mat = Context.material(torch.full((ctx.E,), mu, dtype=torch.float64, device="cuda"),
                               torch.full((ctx.E,), lam, dtype=torch.float64, device="cuda"), pf.RHO)
        (u, newton, pcg), ms = timed(lambda: pf.wave_newmark(
            ctx, mat, T / nsteps, nsteps, FP64, newton_rtol=1e-10, pcg_rtol=1e-10, name="quartic"))
        err = ctx.l2_error(u, pf.exact_at_gauss_points(ctx, "quartic", T))
        ctx.close()
        return {"P": P, "steps": nsteps, "dt": T / nsteps, "l2_error": [float("%.4g" % e) for e in err],
                "newton": newton, "pcg_per_solve": round(pcg / max(newton, 1), 2),
                "ms_per_step": round(ms / nsteps, 3)}

    space = [run(P, 64) for P in (2, 3, 4, 5, 6)]
    time_ = [run(5, n) for n in (8, 16, 32, 64, 128)]
    for r in space + time_:
        log("quartic %s" % r)
    rates = [time_[i]["l2_error"][0] / time_[i + 1]["l2_error"][0] for i in range(len(time_) - 1)]
    return {"case": "quartic", "space_dt_3.9e-4": space, "time_P5": time_,
            "time_error_ratios_per_halving": [round(x, 3) for x in rates]}


def case_condense(a):
    """Static condensation of the element-interior modes (sdme_condensed_pcg)
    against the full Jacobi-PCG on the same FP64 systems, both to 1e-8:
    the Newmark matrix b1 M + K_T (b1 = 4 / dt^2, dt = 0.1) of the 16x4x4
    cantilever (P = 4) at a seeded state for SDME-H, SDME-M and the nodal basis;
    its explicit mass solve (SDME-M); and the tangent of the 47^3, P = 4
    compression workload at its initial guess with right-hand side -R."""
    import torch

    from paper_2104_13466_amd import inputs
    from paper_2104_13466_amd.sdme import FP64, MASK_BC, Context

    def compare(ctx, mat, b, ulin, shift, mass_only, reps):
        out = {}
        xs = {}
        for name in ("full", "condensed"):
            x = torch.zeros_like(b)
            ts = []
            for r in range(1 + reps):
                x.zero_()
                if name == "full":
                    st, ms = timed(lambda: ctx.jacobi_pcg(mat, FP64, b, x, u_lin=ulin,
                                                          mass_shift=shift, mass_only=mass_only,
                                                          rtol=1e-8))
                else:
                    st, ms = timed(lambda: ctx.condensed_pcg(mat, b, x, u_lin=ulin,
                                                             mass_shift=shift,
                                                             mass_only=mass_only, rtol=1e-8))
                if r:
                    ts.append(ms)
            out[name] = {"iterations": st["iterations"], "ms": round(float(np.median(ts)), 2)}
            xs[name] = x
        out["speedup_condensed"] = round(out["full"]["ms"] / out["condensed"]["ms"], 3)
        out["max_rel_diff"] = ((xs["full"] - xs["condensed"]).abs().max() /
                               xs["full"].abs().max()).item()
        return out

    rows = []
    w = inputs.WORKLOADS["cantilever_p4"]
    lam0, mu0 = inputs.lame(w["E"], w["nu"])
    for kind, mass_only in ((4, False), (2, False), (0, False), (2, True)):
        ctx = Context(w["n"], w["L"], w["P"], basis=kind, dirichlet=w["dirichlet"])
        mu = torch.full((ctx.E,), mu0, dtype=torch.float64, device="cuda")
        lam = torch.full((ctx.E,), lam0, dtype=torch.float64, device="cuda")
        mat = Context.material(mu, lam, w["rho"])
        free = 1.0 - ctx.dirichlet_flags().astype(np.float64)
        u = torch.tensor(free * inputs.random_coeffs(w["seed"], w["n"], w["P"], 1e-3),
                         device="cuda")
        b = torch.tensor(free * inputs.uniform(w["seed"], 3 * ctx.Nn, -1, 1, stream=5),
                         device="cuda")
        r = compare(ctx, mat, b, u, 4.0 / 0.1 ** 2, mass_only, 3)
        r.update(workload="cantilever_p4", basis=KIND_NAMES[kind],
                 system="rho M" if mass_only else "b1 M + K_T, b1 = 400",
                 condensed_dofs=ctx.condensed_sizes()[0], full_free_dofs=int(free.sum()))
        log("condense %s" % r)
        rows.append(r)
        ctx.close()
    wl, ctx, mat, u0 = setup("compress_p4")
    R = torch.zeros_like(u0)
    ctx.internal_force(mat, FP64, u0, R, flags=MASK_BC)
    ctx.axpby(-1.0, R, 0.0, R)
    r = compare(ctx, mat, R, u0, 0.0, False, 1)
    r.update(workload="compress_p4", basis="sdme_h", system="K_T at the initial guess, b = -R",
             condensed_dofs=ctx.condensed_sizes()[0])
    log("condense %s" % r)
    rows.append(r)
    return {"case": "condense", "tolerance": 1e-8, "precision": "fp64", "rows": rows}


def case_ordered(a):
    """Ordered assembly against hardware atomics on the workload: per-launch
    times of the element operators (kernel plus gather), and one Newton
    iteration (PCG to 1e-8, FP64 and mixed) run twice from the same state:
    iteration counts and whether the two solutions agree bit for bit."""
    import torch

    from paper_2104_13466_amd.sdme import FP32, FP64
    out = {"case": "ordered", "workload": a.workload, "modes": {}}
    for ordered in (False, True):
        w, ctx, mat, u0 = setup(a.workload, ordered=ordered)
        rows = kernel_table(ctx, mat, u0)
        mode = {"kernels_ms": {"%s_%s" % (r[0], r[1]): round(r[2], 4) for r in rows},
                "device_block_bytes": ctx.context_bytes()[0]}
        for prec in (FP64, FP32):
            runs = []
            for _ in range(2):
                u = u0.clone()
                R, du = torch.zeros_like(u), torch.zeros_like(u)
                st, ms = timed(lambda: newton_iteration(ctx, mat, prec, u, R, du, 1e-8))
                runs.append((st, ms, u))
            key = "fp64" if prec == FP64 else "mixed"
            mode["newton_" + key] = {
                "iterations": [r[0]["iterations"] for r in runs],
                "ms": [round(r[1], 1) for r in runs],
                "bitwise_equal": bool(torch.equal(runs[0][2], runs[1][2])),
                "max_abs_diff": (runs[0][2] - runs[1][2]).abs().max().item()}
            log("ordered=%s %s %s" % (ordered, key, mode["newton_" + key]))
        out["modes"]["ordered" if ordered else "atomic"] = mode
        ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="compress_p4")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the load-stepped Newton-PCG solve in both precisions")
    ap.add_argument("--fp64-reps", type=int, default=2)
    ap.add_argument("--increments", type=int, default=5)
    # At 47^3, P = 4 the tangent stops being positive definite beyond about
    # 16 % nominal compression (PCG meets negative curvature and Newton
    # stalls near the clamped edges), so the load-stepped solve stops at 15 %.
    ap.add_argument("--solve-compression", type=float, default=0.15)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-table", action="store_true")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only the per-operator launches, 12 mixed PCG iterations and a 1 GiB "
                         "copy (for counter runs)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--case", choices=["sweep", "newmark", "explicit", "adjoint", "params",
                                      "static", "wave", "quartic", "condense", "ordered"],
                    help="print the JSON line of a further measurement instead of the benchmark")
    ap.add_argument("--steps-explicit", type=int, default=2000)
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-sub", type=int, default=24, help=argparse.SUPPRESS)
    a = ap.parse_args()
    if a.cpu_baseline_only:
        # host-only child of the benchmark: no device is touched
        from paper_2104_13466_amd import inputs
        print(json.dumps(cpu_baseline(dict(inputs.WORKLOADS[a.workload]), sub_n=a.cpu_sub)))
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: libsdme has no multi-GPU path (slab partition "
              "+ halo exchange over RCCL is designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2104_13466_amd.sdme import FP32, FP64

    if a.case:
        fn = {"sweep": case_sweep, "newmark": case_newmark, "explicit": case_explicit,
              "adjoint": case_adjoint, "params": case_params, "static": case_static,
              "wave": case_wave, "quartic": case_quartic, "condense": case_condense,
              "ordered": case_ordered}[a.case]
        print(json.dumps(fn(a)), flush=True)
        return
    log("setup %s" % a.workload)
    w, ctx, mat, u0 = setup(a.workload)
    N = 3 * ctx.Nn
    log("mesh %s P=%d: %d DOF, %d elements, %d Gauss points" % (w["n"], w["P"], N, ctx.E, ctx.nqp))
    if a.kernel_table or a.profile_kernels:
        rows = kernel_table(ctx, mat, u0)
        if a.profile_kernels:
            # a few iterations of the mixed PCG (its operator fuses the
            # direction update), then the copy of known size
            from paper_2104_13466_amd.sdme import MASK_BC
            R = torch.zeros(N, dtype=torch.float64, device="cuda")
            du = torch.zeros_like(R)
            ctx.internal_force(mat, FP64, u0, R, flags=MASK_BC)
            ctx.axpby(-1.0, R, 0.0, R)
            ctx.jacobi_pcg(mat, FP32, R, du, u_lin=u0, rtol=a.rtol, maxit=12, check=False)
            torch.cuda.synchronize()
            copy_calibration()
        print(json.dumps({"kernel_table": rows}), flush=True)
        return
    if not a.workload.startswith("compress"):
        # the timed step is a Newton iteration of the compression problem; the
        # other workloads are driven by --case (or timed per operator with
        # --kernel-table)
        print("the Newton-iteration benchmark runs on the compress_p* workloads only",
              file=sys.stderr)
        sys.exit(2)
    u = u0.clone()
    R = torch.zeros(N, dtype=torch.float64, device="cuda")
    du = torch.zeros_like(R)
    # warmup
    for i in range(a.warmup):
        u.copy_(u0)
        st = newton_iteration(ctx, mat, FP32, u, R, du, a.rtol)
        log("warmup %d: pcg its %d outer %d rel %.2e (%.0f ms)" % (i, st["iterations"], st["outer"],
                                                                 st["rel_residual"], st["time_ms"]))
    torch.cuda.synchronize()
    ctx.profile(True)
    applies = 0
    times = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        ts = time.perf_counter()
        u.copy_(u0)
        st = newton_iteration(ctx, mat, FP32, u, R, du, a.rtol)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        applies += st["iterations"] + st["outer"]
        log("step %d: pcg its %d outer %d rel %.2e %.1f ms" % (i, st["iterations"], st["outer"],
                                                             st["rel_residual"], 1e3 * times[-1]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile(False)
    ms_step = 1e3 * elapsed / a.steps
    value = applies * N / elapsed / 1e9
    # dominant kernel: FP32 stored-state tangent action inside the inner PCG
    k_ms = prof["fp32_ms"] / max(prof["fp32_count"], 1)
    # algorithmic bytes of the stored-gradient tangent action: a 9-word
    # gradient state per Gauss point (4 B words), read v and write y (4 B per
    # DOF each).  Reported beside them: the bytes this kernel moves beyond
    # that by design -- the 10th state word (mu - lam ln J) and the fused PCG
    # direction update (r, the inverse diagonal and the previous p read and p
    # written, in place of the read of v)
    bytes_launch = 36 * ctx.nqp + 8 * N
    state_word_bytes = 4 * ctx.nqp
    fused_pcg_bytes = 12 * N
    achieved = bytes_launch / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    # sum-factorised contractions (forward and transposed, 3 components) plus
    # the linearised stress at every Gauss point
    P, Q = w["P"], w["P"] + 2
    nn = P + 1
    flops_launch = ctx.E * (2 * 2 * 3 * (2 * Q * nn ** 3 + 3 * Q * Q * nn * nn + 3 * Q ** 3 * nn)
                            + POINTWISE_FLOPS * Q ** 3)
    tflops = flops_launch / (k_ms * 1e-3) / 1e12
    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "GDOF/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%dx%d hexahedra, P=%d, Q=%d, SDME-H, %d DOF, 20%% "
                               "compression, Newton iteration with mixed FP32/FP64 Jacobi-PCG to "
                               "%.0e" % (a.workload, w["n"][0], w["n"][1], w["n"][2], w["P"],
                                         w["P"] + 2, N, a.rtol),
                   "dofs": N, "elements": ctx.E, "gauss_points": ctx.nqp},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_over_algorithmic": (round(traffic / bytes_launch, 3)
                                                  if traffic else None),
                     "kernel": "k_tangent<4,6,float,state,fused p update> (FP32 stored-state "
                               "tangent action, the PCG operator)",
                     "avg_launch_ms": round(k_ms, 4), "launches": prof["fp32_count"],
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "algorithmic_bytes": "36 B per Gauss point (9-word gradient state) + 8 B "
                                          "per DOF (read v, write y)",
                     "state_word_bytes": state_word_bytes,
                     "fused_pcg_bytes": fused_pcg_bytes,
                     "frac_with_design_bytes": round(
                         (bytes_launch + state_word_bytes + fused_pcg_bytes) /
                         (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "kernel_gdofs": round(N / (k_ms * 1e-3) / 1e9, 2),
                     "alu": {"achieved": round(tflops, 2), "peak": FP32_PEAK, "unit": "TFLOP/s",
                             "frac": round(tflops / FP32_PEAK, 4),
                             "algorithmic_flops_per_launch": flops_launch}},
        "tangent_applies_per_step": applies / a.steps,
    }
    # FP64 PCG vs mixed on the same Newton iteration (same state, same
    # tolerance): one warm-up, then the median of a.fp64_reps timed runs
    uf = u0.clone()
    duf = torch.zeros_like(R)
    t64s = []
    for i in range(1 + a.fp64_reps):
        uf.copy_(u0)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        stf = newton_iteration(ctx, mat, FP64, uf, R, duf, a.rtol)
        torch.cuda.synchronize()
        if i:
            t64s.append(time.perf_counter() - ts)
        log("fp64 newton iteration%s: pcg its %d, %.1f ms" % (
            "" if i else " (warm-up)", stf["iterations"], 1e3 * (time.perf_counter() - ts)))
    t64 = float(np.median(t64s))
    dd = ((uf - u).abs().max() / (uf - u0).abs().max()).item()
    result["newton_iteration"] = {
        "fp64": {"ms": round(1e3 * t64, 1), "pcg_iterations": stf["iterations"],
                 "runs_ms": [round(1e3 * t, 1) for t in t64s]},
        "mixed": {"ms": round(ms_step, 1), "pcg_iterations": applies / a.steps,
                  "runs_ms": [round(1e3 * t, 1) for t in times]},
        "speedup_mixed_vs_fp64": round(1e3 * t64 / ms_step, 3),
        "max_rel_diff_increment_mixed_vs_fp64": dd}
    result["other_kernels"] = mass_roofline(ctx)
    if not a.no_solve:
        result["newton_pcg"] = full_solve(ctx, mat, u0, a)
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(w)
        result["cpu_baseline"]["single_thread"] = cpu_baseline_single(a.workload)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
