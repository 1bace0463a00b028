#!/usr/bin/env python3
"""Benchmark: KLE-CGC parareal solves/s at 1e-8 vs the serial fine solution on one MI355X.

Workload (2D diffusion with a log-normal KL coefficient): 128x128 interior grid, KL
d = 10 (corr 0.3, sigma 1), f = 1, T = 1, N = 64 slices, J = 64 fine backward-Euler
steps, alpha = 1e-4, M = 256 samples, float32-refined fine path, float64 coarse
correction, Hermite gPC degree-3 initial guess.  One step = one parareal_solve of the
whole batch (gPC prediction + all parareal iterations to tol 1e-8), inputs resident
in HBM.  The offline stage (training solutions, snapshot KL, gPC fit) runs before the
timed region and is reported separately.

With --config c4_2d_n128_mlp the same problem is solved on 512 fresh samples from the
learned initial guess (an MLP trained on 4096 serial-fine solutions restricted to a
32x32 grid, BF16 MFMA) and, for comparison, from the gPC guess fitted to the same
training set; `value` is then the MLP-initialised rate.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--config NAME] [--init gpc|mlp|both]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
# algorithmic work per unit of the dominant kernels
FLOPS_PER_PCG_UNKNOWN_IT = 18.0        # 5-point scaled matvec 8, two dots 4, three axpys 6
# red-black reduced system, per grid unknown and iteration: odd-node gather 7 and even-node
# gather 9 (each on half the nodes), two dots 4 and three axpys 6 on the even half
FLOPS_PER_RB_UNKNOWN_IT = 13.0
KC_FINE_RB128 = 6
# float64 refinement of the resident fine kernels, per unknown and residual evaluation (one at the
# start of every implicit step and one after every float32 pass): six float64 vectors — state,
# increment, two face-coefficient arrays and D^{-1/2} read, the increment written
BYTES_PER_FP64_RESIDUAL_EVAL = 48.0
BYTES_PER_COCG_UNKNOWN_IT = 128.0      # complex128 vectors streamed per COCG iteration
# streamed multigrid fine path (grids above 128^2), per unknown, one smoothing sweep, float32
# vectors and scaled couplings counted per pass and system (a pass reads a neighbour once):
#  CG iteration: level-0 V-cycle 67 B (first sweep 16, restriction 17, two post-smoothing half
#  sweeps 17 each) + coarser streamed levels ~28 B + P update 12 + matvec 16 + X/R update 24
#  = 147 B; each implicit step: start 48 B + float64 residual 48 B = 96 B; each float64
#  refinement pass: float32 right-hand side 24 B + float64 update 76 B = 100 B
MG_BYTES_PER_CG_IT, MG_BYTES_PER_STEP, MG_BYTES_PER_PASS = 147.0, 96.0, 100.0
PEAK_FP64_TFLOPS = 78.6
# P1 advection-diffusion fine sweep (banded LU of half-bandwidth W), per unknown and
# backward-Euler step of one slice: mass stencil 7 FMA (14), load 3, forward substitution
# W FMA (2W), back substitution W FMA + 1 scaling (2W + 1) -> 4W + 18 flops; the lane's
# state is read and written once by each substitution -> 32 B
def ade_flops_per_row(W: int) -> float:
    return 4.0 * W + 18.0


ADE_BYTES_PER_ROW = 32.0


# nonlinear sweep (one work-group per system, parallel cyclic reduction over P = 2^q >= n rows),
# per unknown and Newton step: f and its Jacobian row ~20, the Newton row and the update ~10,
# each of the q reduction steps 2 divisions + 6 multiplications + 6 additions (+ the final
# division) -> 30 + 14 q flops
def nl_flops_per_row(n: int) -> float:
    q = max(6, math.ceil(math.log2(n)))
    return 30.0 + 14.0 * q


def code_sha256(path: str) -> str:
    """sha256 of a C++ source with its // comments, trailing blanks and empty lines removed:
    it changes with the code, not with the comments (the sources hold no string literal
    containing //)."""
    import hashlib
    import re
    lines = []
    for line in open(path, encoding="utf-8"):
        line = re.sub(r"//.*", "", line).rstrip()
        if line:
            lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def profiled_traffic(kernel_src: str, profile_json: str, shape: dict = None):
    """HBM bytes per launch from the committed rocprofv3 counter passes, or None if the
    kernel source's code has changed since the counters were taken, or if the launch shape
    (grid size, slices, fine steps, samples, kernel variant, launches) differs from the
    profiled one."""
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", profile_json)))
        sha = code_sha256(os.path.join(ROOT, "paper_2510_26180_amd", "csrc", kernel_src))
    except OSError:
        return None
    if prof.get("fine_hip_code_sha256") != sha:
        return None
    if shape is not None and prof.get("shape") != shape:
        return None
    return (prof["fetch_bytes_per_launch"] + prof["write_bytes_per_launch"]) / 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- CPU leg: the oracle
# Worker processes are forked before this process touches the GPU, each limited to one BLAS
# thread; they import the oracle themselves.
def oracle_workers() -> int:
    """Single-threaded oracle workers: the host cores this process may use, at most 16 (the
    CPU share of one GPU), one left for driving the GPU."""
    return max(1, min(len(os.sched_getaffinity(0)), 16) - 1)


def _oracle_init():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"


def _oracle_faces(w, xi_row):
    from oracle import field
    lam, Phi = field.kl_modes(w.dim, w.n, w.d, w.corr_len, w.sigma)
    return field.synthesize(lam, Phi, xi_row[None, :])[0]


def _oracle_serial_fine(job):
    """The oracle's FP64 serial fine solution of one sample, and its time."""
    w, xi_row = job
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import prop
    with threadpool_limits(1):
        a = _oracle_faces(w, xi_row)
        t0 = time.perf_counter()
        P = prop.Propagators(w.dim, w.n, a, w.T, w.N, w.J, w.forcing)
        ref = prop.serial_fine(P, np.zeros(w.Nx), w.N)
        return ref, time.perf_counter() - t0


def _oracle_two_iterations(job):
    """Two parareal iterations (Algorithm 2, diagonalised CGC) of the oracle on one sample:
    the seconds of the first (which also factorises the shifted systems) and of the second."""
    w, xi_row = job
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import parareal as opar, prop
    with threadpool_limits(1):
        a = _oracle_faces(w, xi_row)
        t0 = time.perf_counter()
        P = prop.Propagators(w.dim, w.n, a, w.T, w.N, w.J, w.forcing)
        opar.parareal_diag(P, w.alpha, np.zeros(w.Nx), np.zeros((w.N, w.Nx)), w.tol, 1, fixed_iters=1)
        t1 = time.perf_counter() - t0
        opar.parareal_diag(P, w.alpha, np.zeros(w.Nx), np.zeros((w.N, w.Nx)), w.tol, 2, fixed_iters=2)
        t2 = time.perf_counter() - t0 - t1
        return t1, max(t2 - t1, 0.0)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pool, P, w, xi, subset, iters_mean):
    """The oracle on the host cores: (i) its FP64 serial fine solution of the seeded subset
    of evaluation samples (the accuracy reference of those samples), (ii) two parareal
    iterations on each of P samples, one per worker.  Oracle solves/s = P / (first iteration +
    (mean GPU iteration count - 1) x later iteration), the whole pool busy."""
    t0 = time.perf_counter()
    refs = pool.map(_oracle_serial_fine, [(w, xi[m]) for m in subset], chunksize=1)
    t_ref = time.perf_counter() - t0
    log(f"oracle serial fine on {len(subset)} samples: {t_ref:.1f} s with {P} workers")
    rows = [xi[int(m) % len(xi)] for m in range(P)]
    t0 = time.perf_counter()
    its = pool.map(_oracle_two_iterations, [(w, r) for r in rows], chunksize=1)
    t_its = time.perf_counter() - t0
    t_first = sum(t for t, _ in its) / len(its)
    t_next = sum(t for _, t in its) / len(its)
    t_solve = t_first + max(iters_mean - 1.0, 0.0) * t_next
    log(f"oracle parareal: first iteration {t_first:.1f} s, later {t_next:.1f} s per sample ({t_its:.1f} s wall)")
    base = {"value": P / t_solve, "unit": "solves/s", "cores": P, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{P} samples x 2 parareal iterations ({w.N} slices x {w.J} BE steps + diagonalised CGC), "
                      f"one per single-threaded worker: first {t_first:.1f} s, later {t_next:.1f} s per iteration; "
                      f"a solve = first + ({iters_mean:.2f} - 1) later iterations (mean GPU count)",
            "serial_fine_solves_per_s": len(subset) / t_ref, "serial_fine_sample": f"{len(subset)} samples, "
            f"{t_ref:.1f} s wall on {P} workers (the accuracy reference of the oracle subset)"}
    return base, [r for r, _ in refs]


def run_ragged(args):
    """Ragged batch (uneven grid sizes and slice counts): one parareal_solve_batch call,
    iterations captured into a HIP graph; per-solve latency p50/p99 from the device clock."""
    import numpy as np
    import torch

    import paper_2510_26180_amd as K
    import workloads as W
    spec = W.C3_RAGGED
    bw = spec.base
    grids = tuple(int(g) for g in args.grids.split(",")) if args.grids else spec.grids
    M = args.M or bw.M
    ns, Ns = W.draw_ragged(M, bw.seed_eval, grids, spec.slices)
    xi = W.draw_xi(M, bw.d, bw.seed_eval + 1000)
    dev = torch.device("cuda:0")
    ctx = K.Context(0)
    log(f"ragged batch: M={M}, grids {grids}, slices {spec.slices}, J={bw.J}, alpha={bw.alpha}")
    fc = [2 * int(n) * (int(n) + 1) for n in ns]
    sz = [int(N) * int(n) * int(n) for n, N in zip(ns, Ns)]
    fo = np.concatenate([[0], np.cumsum(fc)[:-1]]).astype(np.int64)
    so = np.concatenate([[0], np.cumsum(sz)[:-1]]).astype(np.int64)
    a_d = torch.empty(int(sum(fc)), dtype=torch.float64, device=dev)
    U = torch.empty(int(sum(sz)), dtype=torch.float64, device=dev)
    base = K.ProblemSpec.from_workload(bw.replace(n=grids[0], N=spec.slices[0]))
    classes = {}
    for m in range(M):
        classes.setdefault((int(ns[m]), int(Ns[m])), []).append(m)
    t0 = time.perf_counter()
    faces = {}
    for g in grids:
        idx = [m for m in range(M) if ns[m] == g]
        if not idx:
            continue
        fh = ctx.kle_build_field(2, g, bw.d, bw.corr_len, bw.sigma)
        ac = torch.empty((len(idx), 2 * g * (g + 1)), dtype=torch.float64, device=dev)
        ctx.kle_synthesize(fh, torch.as_tensor(xi[idx]).to(dev), ac)
        for j, m in enumerate(idx):
            a_d[fo[m]:fo[m] + fc[m]] = ac[j]
        faces[g] = ac
        if not args.no_autotune:
            pg = K.ProblemSpec.from_workload(bw.replace(n=g, N=max(Ns[idx])))
            log(f"autotune n={g}: {ctx.autotune(pg, ac[:4].contiguous())}")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    tasks = [(int(ns[m]), int(Ns[m]), int(fo[m]), int(so[m])) for m in range(M)]
    # accuracy reference: the GPU serial fine solution of every class, computed once
    t0 = time.perf_counter()
    refs = {}
    for (n, N), idx in classes.items():
        pc = K.ProblemSpec.from_workload(bw.replace(n=n, N=N))
        ac = torch.stack([a_d[fo[m]:fo[m] + fc[m]] for m in idx])
        refs[(n, N)] = torch.empty((len(idx), N, n * n), dtype=torch.float64, device=dev)
        ctx.serial_fine_propagate(pc, ac, None, refs[(n, N)])
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0

    def errors():
        e = np.zeros(M)
        for (n, N), idx in classes.items():
            for j, m in enumerate(idx):
                got = U[so[m]:so[m] + sz[m]].view(N, n * n)
                ref = refs[(n, N)][j]
                e[m] = float((got - ref).abs().max() / ref.abs().max())
        return e

    # the per-class graph driver (the default), its eager form, and the persistent fine launch
    modes = [("graph", dict(graph=True))]
    if args.compare_eager:
        modes.append(("eager", dict(graph=False)))
    if args.compare_persistent:
        modes.append(("persistent", dict(graph=True, persistent=True)))
    runs = {}
    for name, kw in modes:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, st, lat, total, rc = ctx.parareal_solve_batch(base, tasks, a_d, U, init=K.KC_INIT_COARSE,
                                                           allow_noconv=True, progress=True, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        runs[name] = dict(its=its, st=st, lat=lat, total=total, wall=wall, rc=rc, err=errors(),
                          fine_ms=ctx.last_times()["fine"][0])
        log(f"{name}: {wall:.2f} s, iterations mean {its.mean():.2f} max {its.max()}, "
            f"latency p50 {np.percentile(lat, 50) / 1e3:.2f} s p99 {np.percentile(lat, 99) / 1e3:.2f} s")
    err = runs["graph"]["err"]
    r = runs["graph"]
    n_ok = int((err <= 1e-8).sum())
    cls_stats = {f"{n}x{n},N={N}": {"samples": len(idx), "iters_mean": float(r["its"][idx].mean()),
                                    "latency_p50_ms": float(np.percentile(r["lat"][idx], 50))}
                 for (n, N), idx in sorted(classes.items())}
    line = {
        "metric": "parareal solves/s at 1e-8 vs serial fine (ragged batch)",
        "value": n_ok / r["wall"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * r["wall"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"c3_ragged: 2D grids {grids} x N {spec.slices}, J={bw.J}, KL d={bw.d}, "
                               f"alpha={bw.alpha}, M={M}, coarse-sweep guess, one parareal_solve_batch "
                               "(HIP-graph iterations)", "samples": M},
        "latency_ms": {"p50": float(np.percentile(r["lat"], 50)), "p99": float(np.percentile(r["lat"], 99)),
                       "max": float(r["lat"].max())},
        "iters": {"mean": float(r["its"].mean()), "max": int(r["its"].max()), "min": int(r["its"].min())},
        "accuracy": {"n_within_1e-8": n_ok, "max_rel_err_vs_serial_fine": float(err.max())},
        "classes": cls_stats, "setup_s": t_setup, "serial_fine_reference_s": t_ref,
    }
    for name in ("eager", "persistent"):
        if name not in runs:
            continue
        e = runs[name]
        line[name] = {"ms": 1e3 * e["wall"], "solves_per_s": int((e["err"] <= 1e-8).sum()) / e["wall"],
                      "latency_p50_ms": float(np.percentile(e["lat"], 50)),
                      "latency_p99_ms": float(np.percentile(e["lat"], 99)),
                      "fine_kernel_ms": e["fine_ms"], "n_within_1e-8": int((e["err"] <= 1e-8).sum()),
                      "max_rel_err_vs_serial_fine": float(e["err"].max()),
                      "same_iterations": bool((e["its"] == r["its"]).all()),
                      "classes": {f"{n}x{n},N={N}": {"iters_mean": float(e["its"][idx].mean()),
                                                     "latency_p50_ms": float(np.percentile(e["lat"][idx], 50))}
                                  for (n, N), idx in sorted(classes.items())}}
    print(json.dumps(line), flush=True)
    ctx.close()


def run_iterations(args):
    """The large configuration (2D 512^2, KL d = 20, N = 256, J = 128, M = 64): a bounded
    number of parareal iterations from the coarse-sweep guess, timed; a full solve (about ten
    iterations) takes over an hour on one GPU, so the line reports the iteration rate."""
    import numpy as np
    import torch

    import paper_2510_26180_amd as K
    import workloads as W
    w = W.get(args.config)
    M = args.M or w.M
    iters = max(1, args.iters)
    dev = torch.device("cuda:0")
    ctx = K.Context(0)
    prob = K.ProblemSpec.from_workload(w, max_iter=iters)
    # one smoothing sweep per level (faster per solve than two at this grid, measured)
    ctx.set_tuning(w.n, fine_variant=5, fine_pcg_rtol=1e-6, cgc_variant=5, cgc_inner_rtol=1e-4, mg_sweeps=1)
    log(f"workload {w.name}: n={w.n} N={w.N} J={w.J} M={M} d={w.d}, {iters} parareal iteration(s)")
    fh = ctx.kle_build_field(2, w.n, w.d, w.corr_len, w.sigma)
    xi = torch.as_tensor(W.draw_xi(M, w.d, w.seed_eval)).to(dev)
    a = torch.empty((M, w.n_faces), dtype=torch.float64, device=dev)
    ctx.kle_synthesize(fh, xi, a)
    U = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.coarse_propagate(prob, a, None, U)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    log(f"coarse-sweep guess: {t_init:.1f} s")
    t0 = time.perf_counter()
    its, st, hist, rc = ctx.parareal_solve(prob, a, U, init=K.KC_INIT_GIVEN, init_U=U, allow_noconv=True)
    torch.cuda.synchronize()
    t_it = time.perf_counter() - t0
    kt = ctx.last_times()
    stats = ctx.last_stats()
    fine_ms, fine_n = kt["fine"]
    byts = w.Nx * (MG_BYTES_PER_CG_IT * stats["fine_krylov_its"] + MG_BYTES_PER_STEP * stats["fine_solves"] +
                   MG_BYTES_PER_PASS * stats["fine_passes"])
    achieved = byts / (fine_ms / 1e3) / 1e9
    deltas = hist[:, :iters]
    line = {
        "metric": "parareal iteration rate, large configuration (not converged: bounded run)",
        "value": M * iters / t_it, "unit": "sample-iterations/s", "n_gpus": 1, "steps": iters, "warmup": 0,
        "ms_per_step": 1e3 * t_it / iters, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: 2D diffusion {w.n}x{w.n}, KL d={w.d} (corr {w.corr_len}, sigma {w.sigma}), "
                               f"N={w.N}, J={w.J}, alpha={w.alpha}, M={M}, coarse-sweep guess, {iters} iteration(s)",
                   "samples": M, "grid": w.n, "slices": w.N, "fine_steps": w.J},
        "init_s": t_init, "iteration_s": t_it / iters,
        "increment_after_iteration": {"median": float(np.median(deltas[:, -1])), "max": float(deltas[:, -1].max())},
        "kernel_ms": {k: v[0] for k, v in kt.items()}, "solver_stats": stats,
        "roofline": {"kernel": "fine multigrid (streamed passes)", "bound": "hbm", "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "algorithmic_gb_per_launch": byts / 1e9 / max(fine_n, 1), "launches": fine_n,
                     "ms_per_launch": fine_ms / max(fine_n, 1),
                     "algorithmic_unit": "147 B per unknown per CG iteration + 96 B per implicit step + 100 B per "
                                         "float64 pass"},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def _oracle_model_run(job):
    """The oracle on one Section 5 sample: serial fine solution and k parareal iterations
    (Algorithm 2 from the zero guess); returns (reference, seconds of the parareal run)."""
    w, c, k = job
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import ade, fem, nonlinear as onl
    with threadpool_limits(1):
        if w.model == 1:
            P = ade.ADEPropagators(fem.Discretisation(w.n, w.beta), c, w.T, w.N, w.J)
            ref = ade.serial_fine(P, P.disc.u0)
            t0 = time.perf_counter()
            ade.parareal_diag(P, w.alpha, P.disc.u0, np.zeros((w.N, w.Nx)), 0.0, k)
        else:
            P = onl.NLPropagators(w.model, w.n, c, w.T, w.N, w.J)
            u0 = P.prob.initial_value()
            ref = onl.serial_fine(P, u0)
            t0 = time.perf_counter()
            onl.parareal_diag(P, w.alpha, u0, np.zeros((w.N, w.Nx)), 0.0, k)
        return ref, time.perf_counter() - t0


MODEL_NAMES = {1: "P1-FEM advection-diffusion", 2: "Burgers (upwind)", 3: "Allen-Cahn"}
# iteration counts Section 5 prints (Section 5.1 only; 5.2 and 5.3 show curves)
PAPER_COUNTS = {1: {"kle_pcgc": 10, "parareal_random": 18, "diag_cgc_random": 18}}


def iterations_to(curve, tol):
    """First k with max over slices of the mean error <= tol (None if never)."""
    for k, e in enumerate(curve):
        if e <= tol:
            return k
    return None


def run_model(args):
    """A Section 5 example: the replication runs (standard parareal and diagonalised CGC from the
    random guess, KLE-PCGC from the KL/gPC guess; mean error against the serial fine solution
    per iteration) and the timed KLE-PCGC batch."""
    import workloads as W
    w = W.MODELS[args.config]
    if args.M:
        w = w.replace(M=args.M)
    pool, P = None, 0
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        P = args.oracle_workers or oracle_workers()
        pool = mp.get_context("fork").Pool(P, initializer=_oracle_init)   # before any GPU call
    import numpy as np
    import torch
    import paper_2510_26180_amd as K
    dev = torch.device("cuda:0")
    ctx = K.Context(0)
    ms = K.ModelSpec(w.model, w.n, w.T, w.N, w.J, w.alpha, tol=0.0, max_iter=w.max_iter, beta=w.beta)
    log(f"model {w.name}: n={w.n} N={w.N} J={w.J} alpha={w.alpha} M={w.M} n_t={w.n_train}")
    _, c_tr, z_tr = W.draw_model_params(w, w.n_train, w.seed_train)
    _, c_ev, z_ev = W.draw_model_params(w, w.M, w.seed_eval)
    c_tr, z_tr = torch.as_tensor(c_tr).to(dev), torch.as_tensor(z_tr).to(dev)
    c_ev_np = c_ev
    c_ev, z_ev = torch.as_tensor(c_ev).to(dev), torch.as_tensor(z_ev).to(dev)
    basis = K.KC_GPC_HERMITE if w.model == K.KC_MODEL_ALLEN_CAHN else K.KC_GPC_LEGENDRE
    # offline: training solutions, snapshot KL, gPC fit
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = torch.empty((w.n_train, w.N, w.Nx), dtype=torch.float64, device=dev)
    ctx.model_serial_fine(ms, c_tr, S)
    kl = ctx.kle_build(S.view(w.n_train, -1), w.eps_kl)
    gpc = ctx.gpc_fit(kl, z_tr, w.gpc_degree, basis=basis)
    torch.cuda.synchronize()
    t_off = time.perf_counter() - t0
    log(f"offline: {w.n_train} training solutions, KL modes {kl.n_modes}, gPC P={gpc.P}: {t_off:.2f} s")
    # reference: the serial fine solution of every evaluation sample (also the time-serial baseline)
    ref = torch.empty((w.M, w.N, w.Nx), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.model_serial_fine(ms, c_ev, ref)
    torch.cuda.synchronize()
    t_serial = time.perf_counter() - t0
    U = torch.empty_like(ref)
    runs = {}
    for name, kw in (("parareal_random", dict(init=K.KC_INIT_RANDOM, seed=w.seed_eval, sequential=True)),
                     ("diag_cgc_random", dict(init=K.KC_INIT_RANDOM, seed=w.seed_eval)),
                     ("kle_pcgc", dict(init=K.KC_INIT_GPC, gpc=gpc, xi=z_ev))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, st, hist, errs = ctx.model_parareal_solve(ms, c_ev, U, ref=ref, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mean_err = errs.mean(axis=0).max(axis=1)          # max over slices of the sample mean
        k_star = iterations_to(mean_err, w.err_tol)
        runs[name] = {"iterations_to_tol": k_star, "mean_error_by_iteration": [float(e) for e in mean_err],
                      "seconds_for_max_iter": dt}
        log(f"{name}: mean error below {w.err_tol:g} at k = {k_star} ({w.max_iter} iterations in {dt:.2f} s)")
    k_kle = runs["kle_pcgc"]["iterations_to_tol"] or w.max_iter
    # timed: KLE-PCGC, every sample k_kle iterations (the Section 5 stop: mean error <= err_tol)
    mt = K.ModelSpec(w.model, w.n, w.T, w.N, w.J, w.alpha, tol=0.0, max_iter=k_kle, beta=w.beta)
    for i in range(args.warmup):
        ctx.model_parareal_solve(mt, c_ev, U, init=K.KC_INIT_GPC, gpc=gpc, xi=z_ev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        its, st, hist, _ = ctx.model_parareal_solve(mt, c_ev, U, init=K.KC_INIT_GPC, gpc=gpc, xi=z_ev)
        log(f"step {i}: {k_kle} iterations on {w.M} samples")
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ms_per_step = 1e3 * t_steps / args.steps
    ktimes = ctx.last_times()
    err = (U - ref).abs().amax(dim=2)                     # [M][N]
    mean_err = float(err.mean(dim=0).max())
    per_sample = err.amax(dim=1).cpu().numpy()
    value = w.M / (ms_per_step / 1e3)
    # roofline of the fine sweep (the dominant kernel)
    stats = ctx.last_stats()
    fine_ms, fine_n = ktimes["fine"]
    secs = fine_ms / 1e3
    if w.model == 1:
        Wb = ((w.n + 1) + 3) // 4 * 4
        systems = w.M * (1 + k_kle * (w.N - 1))
        flops = systems * w.J * w.Nx * ade_flops_per_row(Wb)
        byts = systems * w.J * w.Nx * ADE_BYTES_PER_ROW
        roof = {"kernel": "ade_sweep_kernel", "bound": "alu", "achieved": flops / secs / 1e12,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": flops / secs / 1e12 / PEAK_FP64_TFLOPS,
                "traffic": None, "launches": fine_n, "ms_per_launch": fine_ms / max(fine_n, 1),
                "algorithmic_tflop_per_launch": flops / 1e12 / max(fine_n, 1),
                "algorithmic_unit": f"(4W + 18) flops per unknown, step and slice, W = {Wb}",
                "state_bytes": {"achieved_GB_s": byts / secs / 1e9, "unit": "32 B per unknown, step and slice"},
                "active_lanes": f"{w.N - 1} of 64 (one wavefront per sample, lane = slice)"}
    else:
        newton = stats["fine_krylov_its"]          # Newton steps of all backward-Euler steps
        flops = newton * w.n * nl_flops_per_row(w.n)
        roof = {"kernel": "nl_sweep_kernel", "bound": "alu", "achieved": flops / secs / 1e12,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": flops / secs / 1e12 / PEAK_FP64_TFLOPS,
                "traffic": None, "launches": fine_n, "ms_per_launch": fine_ms / max(fine_n, 1),
                "algorithmic_tflop_per_launch": flops / 1e12 / max(fine_n, 1),
                "algorithmic_unit": f"(30 + 14 q) flops per unknown and Newton step, q = {max(6, math.ceil(math.log2(w.n)))} "
                                    "reduction steps",
                "newton_steps": int(newton), "backward_euler_steps": int(stats["fine_solves"]),
                "newton_per_step": newton / max(stats["fine_solves"], 1),
                "cgc_newton_steps_per_correction": stats["cgc_krylov_its"] / max(w.M * k_kle, 1),
                "cgc_newton_max": int(stats["cgc_max_its"]),
                "backward_euler_steps_at_newton_cap": int(stats["fine_missed"])}
    line = {
        "metric": "parareal solves/s at the Section 5 error threshold vs serial fine",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w.name}: {MODEL_NAMES[w.model]} {w.n if w.model != 1 else f'{w.n}x{w.n}'}, "
                               f"N={w.N}, J={w.J}, alpha={w.alpha}, M={w.M}, "
                               f"{'Hermite' if w.model == 3 else 'Legendre'} gPC p={w.gpc_degree} (n_t={w.n_train})",
                   "samples": w.M, "grid": w.n, "slices": w.N, "fine_steps": w.J},
        "replication": {"criterion": f"max over slices of the mean (over samples) max-norm error <= {w.err_tol:g}",
                        "paper": PAPER_COUNTS.get(w.model), **runs},
        "iterations": k_kle,
        "accuracy": {"mean_error_max_over_slices": mean_err, "max_sample_error": float(per_sample.max()),
                     "n_samples_below_threshold": int((per_sample <= w.err_tol).sum())},
        "serial_fine_gpu": {"solves_per_s": w.M / t_serial, "ms": 1e3 * t_serial},
        "offline_s": t_off,
        "kernel_ms": {k: v[0] for k, v in ktimes.items()},
        "roofline": roof,
    }
    if pool is not None:
        nsub = min(args.oracle_subset, w.M)
        subset = W.draw_subset(w.M, nsub, w.seed_eval + 7)
        jobs = [(w, float(c_ev_np[m]), k_kle) for m in subset]
        t0 = time.perf_counter()
        res = pool.map(_oracle_model_run, jobs, chunksize=1)
        wall = time.perf_counter() - t0
        pool.close()
        t_solve = sum(t for _, t in res) / len(res)
        Rg = ref[subset].cpu().numpy()
        e_ser = [float(np.abs(Rg[j] - r).max() / np.abs(r).max()) for j, (r, _) in enumerate(res)]
        Ug = U[subset].cpu().numpy()
        e_par = [float(np.abs(Ug[j] - r).max()) for j, (r, _) in enumerate(res)]
        line["cpu_baseline"] = {"value": P / t_solve, "unit": "solves/s", "cores": P, "kind": "oracle",
                                "cpu": cpu_model(),
                                "sample": f"{nsub} samples x {k_kle} parareal iterations (Algorithm 2), one per "
                                          f"single-threaded worker, {t_solve:.2f} s each ({wall:.1f} s wall)"}
        line["accuracy"]["oracle_subset"] = {"samples": [int(m) for m in subset],
                                             "max_rel_err_gpu_serial_fine_vs_oracle": max(e_ser),
                                             "max_abs_err_kle_pcgc_vs_oracle_serial_fine": max(e_par)}
        log(f"oracle subset: {line['accuracy']['oracle_subset']}")
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2_2d_n128")
    ap.add_argument("--M", type=int, default=0, help="override the batch size (0 = config)")
    ap.add_argument("--iters", type=int, default=1, help="large configuration: parareal iterations timed")
    ap.add_argument("--n-train", type=int, default=0)
    ap.add_argument("--init", choices=["gpc", "mlp", "both"], default=None,
                    help="initial guess (default: gpc; both for the MLP workload)")
    ap.add_argument("--epochs", type=int, default=0, help="override the MLP epochs (0 = spec)")
    ap.add_argument("--batch", type=int, default=0, help="override the MLP mini-batch (0 = spec)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the built-in kernel choices")
    ap.add_argument("--cgc-rtol", type=float, default=0.0,
                    help="relative residual target of the shifted solves inside parareal_solve (0 = library default)")
    ap.add_argument("--compare-persistent", action="store_true",
                    help="ragged batch: also run the persistent fine launch (KC_BATCH_PERSISTENT)")
    ap.add_argument("--grids", default="", help="ragged batch: comma-separated grid sizes (default 64,128,256)")
    ap.add_argument("--compare-eager", action="store_true", help="ragged batch: also run without the HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline and the oracle accuracy subset)")
    ap.add_argument("--no-oracle-check", action="store_true", help="same as --no-cpu-baseline")
    ap.add_argument("--oracle-subset", type=int, default=16, help="evaluation samples checked against the oracle")
    ap.add_argument("--oracle-workers", type=int, default=0, help="oracle worker processes (0 = host cores, <= 15)")
    args = ap.parse_args()
    args.no_cpu_baseline = args.no_cpu_baseline or args.no_oracle_check
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; sharding the batch over "
                                   "several GPUs is not built"}))
        sys.exit(2)

    if args.config.startswith("f"):
        run_model(args)
        return
    if args.config in ("c3_ragged", "c5_2d_n512"):
        os.environ.setdefault("KLECGC_PROGRESS", "1")   # long calls report from inside the library
    if args.config == "c3_ragged":
        run_ragged(args)
        return
    if args.config == "c5_2d_n512":
        run_iterations(args)
        return

    pool, P = None, 0
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        P = args.oracle_workers or oracle_workers()
        pool = mp.get_context("fork").Pool(P, initializer=_oracle_init)   # before any GPU call

    import numpy as np
    import torch

    import paper_2510_26180_amd as K
    import workloads as W

    w = W.get(args.config)
    if args.M:
        w = w.replace(M=args.M)
    if args.n_train:
        w = w.replace(n_train=args.n_train)
    dev = torch.device("cuda:0")
    ctx = K.Context(0)
    prob = K.ProblemSpec.from_workload(w, cgc_rtol=args.cgc_rtol)
    log(f"workload {w.name}: dim={w.dim} n={w.n} N={w.N} J={w.J} M={w.M} alpha={w.alpha} n_train={w.n_train}")

    # ---- inputs resident in HBM
    field_h = ctx.kle_build_field(w.dim, w.n, w.d, w.corr_len, w.sigma)
    xi_eval_np = W.draw_xi(w.M, w.d, w.seed_eval)
    xi_train_np = W.draw_xi(w.n_train, w.d, w.seed_train)
    xi_eval = torch.as_tensor(xi_eval_np).to(dev)
    xi_train = torch.as_tensor(xi_train_np).to(dev)
    a_eval = torch.empty((w.M, w.n_faces), dtype=torch.float64, device=dev)
    a_train = torch.empty((w.n_train, w.n_faces), dtype=torch.float64, device=dev)
    ctx.kle_synthesize(field_h, xi_eval, a_eval)
    ctx.kle_synthesize(field_h, xi_train, a_train)

    init = args.init or ("both" if "mlp" in w.name else "gpc")
    inits = {"gpc": ["gpc"], "mlp": ["mlp"], "both": ["mlp", "gpc"]}[init]
    spec = W.MLP_C4
    if args.epochs:
        spec = W.MlpSpec(**{**spec.__dict__, "epochs": args.epochs})
    if args.batch:
        spec = W.MlpSpec(**{**spec.__dict__, "batch": args.batch})

    # ---- offline stage (untimed): autotuning, training solutions, snapshot KL + gPC fit, MLP training
    torch.cuda.synchronize()
    tuning = None
    t_tune = 0.0
    if not args.no_autotune and w.dim == 2 and w.precision == "f32_refined":
        t0 = time.perf_counter()
        tuning = ctx.autotune(prob, a_train[:16].contiguous())
        t_tune = time.perf_counter() - t0
        log(f"offline: autotune {t_tune:.1f} s -> {tuning}")
    t0 = time.perf_counter()
    S = torch.empty((w.n_train, w.N * w.Nx), dtype=torch.float64, device=dev)
    ctx.serial_fine_propagate(prob, a_train, None, S.view(w.n_train, w.N, w.Nx))
    torch.cuda.synchronize()
    t_snap = time.perf_counter() - t0
    log(f"offline: {w.n_train} training solutions {t_snap:.1f} s")
    offline = {"autotune_s": t_tune, "training_solutions_s": t_snap}
    gpc = mlp = None
    learned = None
    if "mlp" in inits:
        t1 = time.perf_counter()
        nc = spec.nc
        O = w.N * nc * nc
        Yc = torch.empty((w.n_train, O), dtype=torch.float32, device=dev)
        ctx.grid_restrict(w.n, nc, S, Yc)
        mlp = ctx.mlp_create(w.d, spec.hidden, O, params=torch.as_tensor(
            W.draw_mlp_init(w.d, spec.hidden, O, spec.seed_init)).to(dev))
        ctx.mlp_normalize_targets(mlp, Yc)
        perm = torch.as_tensor(W.draw_perms(spec.epochs, w.n_train, spec.seed_perm)).to(dev)
        losses = ctx.mlp_train(mlp, xi_train, Yc, epochs=spec.epochs, batch=spec.batch, lr=spec.lr, perm=perm,
                               lr_final=spec.lr_final)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        ms_train = ctx.last_times()["mlp"][0]
        H, B, n_in_pad = spec.hidden, spec.batch, (w.d + 15) // 16 * 16
        n_steps = spec.epochs * ((w.n_train + B - 1) // B)
        flops_step = 2.0 * B * (n_in_pad * H + H * H + H * O) + 2.0 * B * (2 * H * O + 2 * H * H + w.d * H)
        tflops = flops_step * n_steps / (ms_train / 1e3) / 1e12
        learned = {"hidden": H, "nc": nc, "outputs": O, "params": mlp.n_params, "epochs": spec.epochs,
                   "batch": B, "lr": spec.lr, "lr_final": spec.lr_final, "adam_steps": n_steps, "loss_first": float(losses[0]),
                   "loss_last": float(losses[-1]), "train_s": t_train, "train_kernel_ms": ms_train,
                   "train_tflops": tflops, "train_frac_bf16_peak": tflops / PEAK_BF16_TFLOPS}
        log(f"offline: MLP {mlp.n_params} params, {spec.epochs} epochs in {t_train:.1f} s "
            f"({tflops:.1f} TFLOP/s), loss {losses[0]:.3e} -> {losses[-1]:.3e}")
        offline["mlp_train_s"] = t_train
        del Yc
    if "gpc" in inits:
        t1 = time.perf_counter()
        kl = ctx.kle_build(S, w.eps_kl)
        gpc = ctx.gpc_fit(kl, xi_train, w.gpc_degree)
        torch.cuda.synchronize()
        offline["kl_gpc_s"] = time.perf_counter() - t1
        log(f"offline: KL modes {kl.n_modes}, gPC P={gpc.P}, {offline['kl_gpc_s']:.1f} s")
    del S
    t_offline = sum(offline.values())

    U = torch.empty((w.M, w.N, w.Nx), dtype=torch.float64, device=dev)

    def step(kind):
        if kind == "mlp":
            ctx.mlp_initial_guess(mlp, w.n, spec.nc, w.N, xi_eval, U)
            return ctx.parareal_solve(prob, a_eval, U, init=K.KC_INIT_GIVEN, init_U=U, allow_noconv=True)
        return ctx.parareal_solve(prob, a_eval, U, init=K.KC_INIT_GPC, gpc=gpc, xi=xi_eval, allow_noconv=True)

    # the seeded subset of evaluation samples checked against the oracle's serial fine solution
    subset = W.draw_subset(w.M, min(args.oracle_subset, w.M), w.seed_eval + 7)
    # accuracy reference: batched GPU serial fine for every evaluation sample
    ref = torch.empty_like(U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.serial_fine_propagate(prob, a_eval, None, ref)
    torch.cuda.synchronize()
    t_serial = time.perf_counter() - t0
    refmax = ref.abs().amax(dim=(1, 2))
    results = {}
    for kind in inits:
        # quality of the initial guess itself (untimed)
        if kind == "mlp":
            ctx.mlp_initial_guess(mlp, w.n, spec.nc, w.N, xi_eval, U)
        else:
            ctx.gpc_predict(gpc, xi_eval, U.view(w.M, -1))
        e0 = ((U - ref).abs().amax(dim=(1, 2)) / refmax).cpu().numpy()
        for i in range(args.warmup):
            its, st, _, _ = step(kind)
            log(f"[{kind}] warmup {i}: iterations mean {its.mean():.2f} max {its.max()}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            its, status, hist, rc = step(kind)
            log(f"[{kind}] step {i}: iterations mean {its.mean():.2f} max {its.max()} rc={rc}")
        torch.cuda.synchronize()
        t_steps = time.perf_counter() - t0
        ktimes = ctx.last_times()
        stats = ctx.last_stats()
        err = ((U - ref).abs().amax(dim=(1, 2)) / refmax).cpu().numpy()
        results[kind] = dict(ms_per_step=1e3 * t_steps / args.steps, its=its, err=err, ktimes=ktimes, e0=e0,
                             stats=stats, U_sub=U[subset].cpu().numpy() if kind == inits[0] else None)
    primary = results[inits[0]]
    ms_per_step, its, err, ktimes, stats = (primary[k] for k in ("ms_per_step", "its", "err", "ktimes", "stats"))
    n_ok = int((err <= 1e-8).sum())
    value = n_ok / (ms_per_step / 1e3)

    # ---- roofline of the dominant kernel (HIP-event time of the last timed step)
    dom = max(ktimes, key=lambda k: ktimes[k][0])
    dom_ms, dom_n = ktimes[dom]
    if dom == "fine":
        fv = (tuning or {}).get("fine_variant", -1)
        if fv < 0:   # the library's built-in choice by grid size
            fv = KC_FINE_RB128 if 64 < w.n <= 128 else -1
        per_it = FLOPS_PER_RB_UNKNOWN_IT if fv == KC_FINE_RB128 else FLOPS_PER_PCG_UNKNOWN_IT
        flops = per_it * w.Nx * stats["fine_krylov_its"]
        evals = stats["fine_passes"] + stats["fine_solves"]   # float64 residual evaluations
        byts = BYTES_PER_FP64_RESIDUAL_EVAL * w.Nx * evals
        secs = dom_ms / 1e3
        shape = {"n": w.n, "N": w.N, "J": w.J, "M": w.M, "variant": fv, "launches": dom_n}
        traffic = profiled_traffic("fine.hip", "fine2d_resident_c2_traffic.json", shape)
        ms_launch = dom_ms / max(dom_n, 1)
        fine_hbm = None if traffic is None else {
            "GB_per_s": traffic / (ms_launch / 1e3), "frac_of_peak": traffic / (ms_launch / 1e3) / PEAK_HBM_GBS,
            "source": "profiled FETCH_SIZE + WRITE_SIZE bytes per launch / live launch time"}
        achieved = byts / secs / 1e9
        roof = {"kernel": "fine2d_resident_kernel", "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                "traffic": traffic,
                "traffic_unit": "GB/launch (HBM FETCH+WRITE, copy-calibrated)",
                "algorithmic_gb_per_launch": byts / 1e9 / max(dom_n, 1),
                "algorithmic_unit": "48 B per unknown per float64 residual evaluation",
                "launches": dom_n, "ms_per_launch": ms_launch, "fine_prop_hbm": fine_hbm,
                "krylov_alu": {"solver": "red-black reduced CG" if fv == KC_FINE_RB128 else "Jacobi PCG",
                               "achieved_tflops": flops / secs / 1e12, "peak_tflops": PEAK_FP32_TFLOPS,
                               "frac": flops / secs / 1e12 / PEAK_FP32_TFLOPS,
                               "algorithmic_tflop_per_launch": flops / 1e12 / max(dom_n, 1)}}
    elif dom == "shifted":
        byts = BYTES_PER_COCG_UNKNOWN_IT * w.Nx * stats["cgc_krylov_its"]
        achieved = byts / (dom_ms / 1e3) / 1e9
        roof = {"kernel": "cocg_kernel", "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "launches": dom_n, "ms_per_launch": dom_ms / max(dom_n, 1)}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": None, "traffic": None}

    line = {
        "metric": "parareal solves/s at 1e-8 vs serial fine",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: 2D diffusion {w.n}x{w.n}, KL d={w.d}, N={w.N}, J={w.J}, "
                               f"alpha={w.alpha}, M={w.M}, gPC p={w.gpc_degree} (n_t={w.n_train})",
                   "samples": w.M, "grid": w.n, "slices": w.N, "fine_steps": w.J},
        "iters": {"mean": float(its.mean()), "max": int(its.max()), "min": int(its.min()),
                  "hist": {int(k): int(v) for k, v in zip(*np.unique(its, return_counts=True))}},
        "accuracy": {"n_within_1e-8": n_ok, "reference": "batched GPU serial fine (float64 residuals to 1e-13)",
                     "max_rel_err_vs_serial_fine": float(err.max()), "median_rel_err": float(np.median(err))},
        "serial_fine_gpu": {"solves_per_s": w.M / t_serial, "ms": 1e3 * t_serial},
        "offline_s": t_offline,
        "offline": offline,
        "kernel_ms": {k: v[0] for k, v in ktimes.items()},
        "solver_stats": stats,
        "tuning": tuning,
        "roofline": roof,
    }
    line["init"] = inits[0]
    if learned is not None:
        line["learned"] = learned
    if len(inits) > 1:
        line["compare"] = {k: {"solves_per_s": int((r["err"] <= 1e-8).sum()) / (r["ms_per_step"] / 1e3),
                               "ms_per_step": r["ms_per_step"], "iters_mean": float(r["its"].mean()),
                               "iters_max": int(r["its"].max()),
                               "hist": {int(a): int(b) for a, b in zip(*np.unique(r["its"], return_counts=True))},
                               "n_within_1e-8": int((r["err"] <= 1e-8).sum()),
                               "max_rel_err": float(r["err"].max()),
                               "init_err_median": float(np.median(r["e0"])), "init_err_max": float(r["e0"].max())}
                           for k, r in results.items()}
    if pool is not None:
        log(f"oracle leg: serial fine on {len(subset)} evaluation samples and the CPU baseline, {P} workers")
        base, refs = cpu_baseline(pool, P, w, xi_eval_np, subset, float(its.mean()))
        pool.close()
        line["cpu_baseline"] = base
        Ug = primary["U_sub"]
        Rg = ref[subset].cpu().numpy()
        e_par = [float(np.abs(Ug[j] - r).max() / np.abs(r).max()) for j, r in enumerate(refs)]
        e_ser = [float(np.abs(Rg[j] - r).max() / np.abs(r).max()) for j, r in enumerate(refs)]
        line["accuracy"]["oracle_subset"] = {
            "samples": [int(m) for m in subset], "n_within_1e-8": int(sum(e <= 1e-8 for e in e_par)),
            "max_rel_err_parareal_vs_oracle_serial_fine": max(e_par),
            "max_rel_err_gpu_serial_fine_vs_oracle": max(e_ser)}
        log(f"oracle subset: {line['accuracy']['oracle_subset']}")
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
