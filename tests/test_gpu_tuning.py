"""GPU parity of every kernel variant the autotuner may choose, forced through
klecgc_set_tuning, against the oracle; and the autotuner itself.

The variants differ only in how the Krylov solves are laid out on the GPU (resident in
a work-group or streamed through device memory, float32 or float64 inner loop) and in
the float32 reduction asked of each refinement pass; the float64 residual targets that
end every solve are the same, so each variant must meet the same bound.
"""
import numpy as np
import pytest

import workloads as W
from oracle import cgc, parareal as opar, prop
from tests.gpu_helpers import dev, host, log, oracle_faces, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FINE = {"stream64": 0, "res16": 1, "res32": 2, "res64": 3, "res128": 4, "mg": 5, "rb128": 6}
CGC = {"stream64": 0, "res16": 1, "res32": 2, "res64": 3, "stream32": 4, "mg32": 5}


@pytest.fixture()
def ctx():
    import paper_2510_26180_amd as K
    c = K.Context(0)
    yield c
    c.close()


def spec_of(w, **kw):
    from paper_2510_26180_amd import ProblemSpec
    return ProblemSpec.from_workload(w, **kw)


@pytest.mark.parametrize("n,variant,rtol", [(13, "res16", 1e-5), (13, "res32", 3e-7), (13, "res64", 1e-6),
                                            (13, "res128", 1e-6), (13, "stream64", 1e-6), (20, "res32", 3e-6),
                                            (40, "res64", 1e-5), (40, "res128", 3e-7), (100, "res128", 1e-5),
                                            (1, "mg", 1e-5), (13, "mg", 1e-6), (40, "mg", 1e-5), (100, "mg", 3e-6),
                                            (150, "mg", 1e-5), (132, "mg", 3e-6), (150, "stream64", 1e-6),
                                            # red-black reduced system: odd and even n, padding
                                            # rows and lanes, one node, the full 128 tile
                                            (1, "rb128", 1e-6), (13, "rb128", 1e-6), (40, "rb128", 3e-7),
                                            (100, "rb128", 1e-5), (101, "rb128", 1e-6), (128, "rb128", 3e-6)])
def test_fine_variants(ctx, n, variant, rtol):
    log(f"fine variant {variant} n={n} pass reduction {rtol}")
    # multigrid smoothing: Gauss-Seidel (default) except damped Jacobi at n = 40
    ctx.set_tuning(n, fine_variant=FINE[variant], fine_pcg_rtol=rtol, mg_sweeps=1 if n == 100 else 0,
                   mg_smoother=1 if n == 40 else 0)
    w = W.small_2d(n=n, N=4, J=16)
    M = 2
    xi = W.draw_xi(M, w.d, 41)
    a = oracle_faces(w, xi)
    starts = W.draw_uniform((M, w.N, w.Nx), 42) * 0.05
    end = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    ctx.fine_propagate(spec_of(w, precision=1, inner_rtol=1e-14), dev(a), dev(starts), end)
    got = host(end)
    for m in range(M):
        P = prop.Propagators(2, n, a[m], w.T, w.N, w.J, w.forcing)
        for s in range(w.N):
            assert rel(got[m, s], P.F(starts[m, s])) < 1e-11


@pytest.mark.parametrize("n,variant,rtol", [(13, "res16", 1e-4), (13, "res32", 1e-5), (13, "res64", 3e-6),
                                            (13, "stream32", 1e-5), (13, "stream64", 1e-5), (40, "res64", 3e-5),
                                            (40, "stream32", 1e-4), (100, "stream32", 3e-6),
                                            (100, "stream64", 1e-5), (1, "mg32", 1e-5), (2, "mg32", 1e-5),
                                            (13, "mg32", 1e-4), (40, "mg32", 1e-5), (100, "mg32", 3e-6),
                                            (128, "mg32", 3e-5)])
def test_cgc_variants(ctx, n, variant, rtol):
    log(f"shifted-solve variant {variant} n={n} pass reduction {rtol}")
    # multigrid smoothing: Gauss-Seidel (default) except damped Jacobi at n = 100
    ctx.set_tuning(n, cgc_variant=CGC[variant], cgc_inner_rtol=rtol, mg_sweeps=1 if n in (40, 128) else 0,
                   mg_smoother=1 if n == 100 else 0)
    N, alpha = 8, 1e-4
    w = W.small_2d(n=n, N=N, alpha=alpha)
    M = 2
    xi = W.draw_xi(M, w.d, 43)
    a = oracle_faces(w, xi)
    r = W.draw_normal((M, N, w.Nx), 44)
    u = torch.empty_like(dev(r))
    ctx.cgc_diag_solve(spec_of(w, precision=1, cgc_rtol=1e-14), dev(a), dev(r), u, allow_noconv=True)
    got = host(u)
    amp = alpha ** (-(N - 1) / N)
    for m in range(M):
        assert rel(got[m], cgc.diag_solve(2, n, a[m], w.T / N, alpha, r[m])) < max(1e-10, 1e-13 * amp)


def test_tuning_rejects_variants_that_do_not_fit(ctx):
    import paper_2510_26180_amd as K
    for kw in (dict(fine_variant=FINE["res32"]), dict(cgc_variant=CGC["res64"]), dict(fine_pcg_rtol=0.0),
               dict(fine_variant=7)):
        with pytest.raises(K.KlecgcError) as e:
            ctx.set_tuning(100, **kw)
        assert e.value.code == -1
    with pytest.raises(K.KlecgcError):
        ctx.set_tuning(100, mg_sweeps=5)
    with pytest.raises(K.KlecgcError):
        ctx.set_tuning(100, mg_smoother=2)
    assert ctx.get_tuning(100) == {"fine_variant": -1, "fine_pcg_rtol": pytest.approx(1e-6),
                                   "cgc_variant": -1, "cgc_inner_rtol": pytest.approx(1e-5), "mg_sweeps": 0,
                                   "mg_smoother": 0}


@pytest.mark.parametrize("n", [20, 72])
def test_autotune_then_parareal_matches_oracle(ctx, n):
    w = W.small_2d(n=n, N=8, J=8, alpha=1e-2, d=6, precision="f32_refined")
    M = 3
    xi = W.draw_xi(M, w.d, 45)
    a = oracle_faces(w, xi)
    prob = spec_of(w)
    t = ctx.autotune(prob, dev(a))
    log(f"  autotune n={n}: {t}")
    assert t["fine_variant"] in (FINE["res32"], FINE["res64"], FINE["res128"], FINE["rb128"]) if n == 20 else \
        t["fine_variant"] in (FINE["res128"], FINE["rb128"])
    assert t["fine_ms"] > 0 and t["cgc_ms"] > 0
    assert ctx.get_tuning(n)["fine_variant"] == t["fine_variant"]
    U = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    its, st, _, _ = ctx.parareal_solve(prob, dev(a), U)
    got = host(U)
    for m in range(M):
        P = prop.Propagators(2, n, a[m], w.T, w.N, w.J, w.forcing)
        assert st[m] == 0
        assert rel(got[m], prop.serial_fine(P, np.zeros(w.Nx), w.N)) <= 1e-8
