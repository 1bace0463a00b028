"""GPU parity: every C-ABI entry point against the CPU oracle, element by element.

Inputs are seeded and synthetic (workloads); expected values come only from the
oracle.  Tolerances: 1e-10 relative for float64 paths (the stated float64 bar), with
the coarse correction's bound scaled by the alpha-circulant round-off growth
alpha^{-(N-1)/N} where stated; iteration counts must be equal.
"""
import numpy as np
import pytest

import workloads as W
from oracle import cgc, gpc as ogpc, parareal as opar, prop, snapshot
from tests.gpu_helpers import dev, host, log, oracle_faces, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_2510_26180_amd as K
    c = K.Context(0)
    yield c
    c.close()


def spec_of(w, **kw):
    from paper_2510_26180_amd import ProblemSpec
    return ProblemSpec.from_workload(w, **kw)


# ---------------------------------------------------------------- field synthesis
@pytest.mark.parametrize("w", [W.get("c1_1d_n127"), W.small_2d(), W.small_2d(n=37, d=10)])
def test_field_synthesis(ctx, w):
    log(f"field synthesis dim={w.dim} n={w.n} d={w.d}")
    xi = W.draw_xi(5, w.d, 99)
    want = oracle_faces(w, xi)
    fh = ctx.kle_build_field(w.dim, w.n, w.d, w.corr_len, w.sigma)
    a = torch.empty((5, w.n_faces), dtype=torch.float64, device="cuda")
    ctx.kle_synthesize(fh, dev(xi), a)
    assert rel(host(a), want) < 1e-12


# ---------------------------------------------------------------- fine propagator
def _fine_case(ctx, w, M, seed, prec_kw):
    xi = W.draw_xi(M, w.d, seed)
    a = oracle_faces(w, xi)
    starts = W.draw_uniform((M, w.N, w.Nx), seed + 1) * 0.05
    prob = spec_of(w, **prec_kw)
    end = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    ctx.fine_propagate(prob, dev(a), dev(starts), end)
    got = host(end)
    worst = 0.0
    for m in range(M):
        P = prop.Propagators(w.dim, w.n, a[m], w.T, w.N, w.J, w.forcing)
        for s in range(w.N):
            worst = max(worst, rel(got[m, s], P.F(starts[m, s])))
    return worst


@pytest.mark.parametrize("n,N,J,M", [(1, 2, 1, 1), (31, 8, 8, 3), (127, 16, 32, 8)])
def test_fine_1d(ctx, n, N, J, M):
    log(f"fine 1D n={n} N={N} J={J} M={M}")
    w = W.small_1d(n=n, N=N, J=J)
    assert _fine_case(ctx, w, M, 5, {}) < 1e-12


@pytest.mark.parametrize("n", [1, 7, 20, 33])
def test_fine_2d_f64(ctx, n):
    log(f"fine 2D f64 n={n}")
    w = W.small_2d(n=n, N=4, J=3)
    assert _fine_case(ctx, w, 2, 7, dict(precision=0, inner_rtol=1e-14)) < 1e-11


@pytest.mark.parametrize("n", [1, 9, 20, 33, 64, 100, 128, 129, 200])
def test_fine_2d_f32_refined(ctx, n):
    log(f"fine 2D f32-refined n={n}")
    w = W.small_2d(n=n, N=4, J=16)   # dt = 1/64, the c2 slice length
    assert _fine_case(ctx, w, 2, 11, dict(precision=1, inner_rtol=1e-14)) < 1e-11


@pytest.mark.parametrize("n,J", [(72, 1), (72, 2), (72, 3), (13, 2), (13, 3), (101, 3), (200, 3)])
def test_fine_2d_f32_refined_few_steps(ctx, n, J):
    # the start of step j is 0 (j = 0), inc_0 (j = 1), then 2 inc_{j-1} - inc_{j-2}: slices of
    # one to three steps cover each rule and the switch between them (resident red-black at 72
    # and 101, full-system resident at 13, multigrid at 200)
    log(f"fine 2D f32-refined n={n} J={J}")
    w = W.small_2d(n=n, N=4, J=J)
    assert _fine_case(ctx, w, 2, 13, dict(precision=1, inner_rtol=1e-14)) < 1e-11


@pytest.mark.parametrize("prec,M,N", [(1, 3, 4), (1, 5, 4), (1, 21, 4), (1, 11, 2), (0, 3, 4)])
def test_fine_2d_work_group_counts(ctx, prec, M, N):
    # systems are numbered XCD-major: with G = M N work-groups not a multiple of 8 (12, 20,
    # 84, 22) the first G mod 8 XCDs take one system more; every (sample, slice) result is still
    # checked against its own start (red-black resident kernel at 72, or float64 PCG)
    log(f"fine 2D prec={prec} n=72 M={M} N={N}")
    w = W.small_2d(n=72, N=N, J=4)
    kw = dict(precision=1, inner_rtol=1e-14) if prec else dict(precision=0, inner_rtol=1e-14)
    assert _fine_case(ctx, w, M, 17, kw) < 1e-11


# ---------------------------------------------------------------- coarse correction
# N = 64, 128 and 256 run their own slice-FFT instances (32, 16 and 8 columns per
# work-group, whose per-sample maxima reduce inside a partial wave); alpha = 1e-4 at large N
# gives the smallest shifts (1 - alpha^{1/N} = 0.035 at N = 256), where step (b) is hardest
@pytest.mark.parametrize("dim,n,N,alpha", [(1, 31, 8, 1e-2), (1, 127, 16, 1e-2), (1, 5, 2, 0.5),
                                           (2, 12, 8, 1e-2), (2, 20, 16, 1e-4), (2, 1, 4, 0.3),
                                           (1, 31, 64, 1e-4), (1, 9, 256, 1e-2), (2, 12, 32, 1e-4),
                                           (2, 12, 64, 1e-4), (2, 12, 128, 1e-4), (2, 12, 256, 1e-4),
                                           (2, 72, 64, 1e-4)])
def test_cgc_diag_solve(ctx, dim, n, N, alpha):
    log(f"cgc dim={dim} n={n} N={N} alpha={alpha}")
    w = (W.small_1d if dim == 1 else W.small_2d)(n=n, N=N, alpha=alpha)
    M = 3
    xi = W.draw_xi(M, w.d, 17)
    a = oracle_faces(w, xi)
    r = W.draw_normal((M, N, w.Nx), 18)
    prob = spec_of(w, cgc_rtol=1e-15, cgc_max_iter=50000)
    u = torch.empty_like(dev(r))
    ctx.cgc_diag_solve(prob, dev(a), dev(r), u, allow_noconv=True)
    got = host(u)
    amp = alpha ** (-(N - 1) / N)
    for m in range(M):
        want = cgc.diag_solve(dim, n, a[m], w.T / N, alpha, r[m])
        assert rel(got[m], want) < max(1e-10, 1e-13 * amp)


@pytest.mark.parametrize("n,N,alpha", [(12, 8, 1e-2), (20, 16, 1e-4), (33, 8, 1e-4), (64, 16, 1e-4), (1, 4, 0.3),
                                     (65, 4, 1e-2), (100, 8, 1e-4), (12, 64, 1e-4), (12, 128, 1e-4),
                                     (12, 256, 1e-4), (72, 64, 1e-4), (128, 64, 1e-4)])
def test_cgc_diag_solve_resident(ctx, n, N, alpha):
    # float32 complex COCG with float64 residual refinement: CU-resident for n <= 64, the
    # multigrid-preconditioned streaming kernel above (n = 128, N = 64 is the c2 shape)
    log(f"cgc resident n={n} N={N} alpha={alpha}")
    w = W.small_2d(n=n, N=N, alpha=alpha)
    M = 2
    xi = W.draw_xi(M, w.d, 19)
    a = oracle_faces(w, xi)
    r = W.draw_normal((M, N, w.Nx), 20)
    prob = spec_of(w, precision=1, cgc_rtol=1e-14)
    u = torch.empty_like(dev(r))
    ctx.cgc_diag_solve(prob, dev(a), dev(r), u, allow_noconv=True)
    got = host(u)
    amp = alpha ** (-(N - 1) / N)
    for m in range(M):
        want = cgc.diag_solve(2, n, a[m], w.T / N, alpha, r[m])
        assert rel(got[m], want) < max(1e-10, 1e-13 * amp)


@pytest.mark.parametrize("dim,n", [(1, 31), (2, 12)])
def test_coarse_propagate(ctx, dim, n):
    log(f"coarse sweep dim={dim} n={n}")
    w = (W.small_1d if dim == 1 else W.small_2d)(n=n)
    M = 2
    xi = W.draw_xi(M, w.d, 23)
    a = oracle_faces(w, xi)
    U = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    ctx.coarse_propagate(spec_of(w, inner_rtol=1e-14), dev(a), None, U)
    got = host(U)
    for m in range(M):
        P = prop.Propagators(dim, n, a[m], w.T, w.N, w.J, w.forcing)
        assert rel(got[m], prop.coarse_sweep(P, np.zeros(w.Nx), w.N)) < 1e-11


# ---------------------------------------------------------------- parareal driver
def _parareal_case(ctx, w, M, init_name, prec_kw, seed=31):
    import paper_2510_26180_amd as K
    xi = W.draw_xi(M, w.d, seed)
    a = oracle_faces(w, xi)
    prob = spec_of(w, **prec_kw)
    U = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    init = {"zero": K.KC_INIT_ZERO, "coarse": K.KC_INIT_COARSE}[init_name]
    iters, status, hist, _ = ctx.parareal_solve(prob, dev(a), U, init=init)
    got = host(U)
    out = []
    for m in range(M):
        P = prop.Propagators(w.dim, w.n, a[m], w.T, w.N, w.J, w.forcing)
        u0 = np.zeros(w.Nx)
        U0 = np.zeros((w.N, w.Nx)) if init_name == "zero" else prop.coarse_sweep(P, u0, w.N)
        h = opar.parareal_diag(P, w.alpha, u0, U0, w.tol, w.max_iter)
        ref = prop.serial_fine(P, u0, w.N)
        out.append((int(iters[m]), h.iters, rel(got[m], h.iterates[-1]), rel(got[m], ref), int(status[m]),
                    hist[m, :iters[m]], h.deltas))
    return out


@pytest.mark.parametrize("init", ["zero", "coarse"])
def test_parareal_1d_c1(ctx, init):
    w = W.get("c1_1d_n127")
    log(f"parareal c1 init={init}")
    for it_gpu, it_or, e_or, e_ref, st, hg, ho in _parareal_case(ctx, w, w.M, init, {}):
        assert st == 0
        assert it_gpu == it_or
        assert e_or < 1e-10
        assert e_ref < 1e-8
        assert np.allclose(hg, ho, rtol=1e-5, atol=1e-13)


def iterations_agree(it_gpu: int, it_or: int, deltas_or, tol: float) -> bool:
    """Equal iteration counts, or one apart when the oracle's increment at the deciding
    iteration lies within 1% of tol (both sides then stop on a rounding-level difference)."""
    if it_gpu == it_or:
        return True
    if it_gpu == it_or - 1 and it_or >= 2:
        return deltas_or[it_or - 2] <= 1.01 * tol
    if it_gpu == it_or + 1:
        return deltas_or[it_or - 1] >= 0.99 * tol
    return False


@pytest.mark.parametrize("prec,n", [(0, 12), (0, 33), (1, 12), (1, 72), (1, 130)])
def test_parareal_2d_small(ctx, prec, n):
    # n = 72: resident fine kernel + multigrid COCG; n = 130: multigrid fine kernel too.
    # float64 (prec 0): equal iteration counts and the oracle's Alg. 2 iterate to 1e-10;
    # float32-refined: iterates to 1e-8 (the float32 Krylov passes stop at their own
    # residual targets, so the paths agree to the refinement tolerance, not to round-off)
    w = W.small_2d(n=n, N=8 if n < 100 else 4, J=6 if n < 100 else 3, alpha=1e-2)
    log(f"parareal 2D small prec={prec} n={n}")
    for it_gpu, it_or, e_or, e_ref, st, hg, ho in _parareal_case(
            ctx, w, 3 if n < 100 else 1, "zero", dict(precision=prec, inner_rtol=1e-14, cgc_rtol=1e-14)):
        assert st == 0
        assert e_ref < 1e-8
        if prec == 0:
            assert it_gpu == it_or
            assert e_or < 1e-10
            assert np.allclose(hg, ho, rtol=1e-6, atol=1e-13)
        else:
            assert iterations_agree(it_gpu, it_or, ho, w.tol)
            assert e_or < 1e-8


@pytest.mark.parametrize("J,M", [(2, 1), (4, 1)])
def test_parareal_c2_shape(ctx, J, M):
    # the c2 grid, slice count and twist (128^2, N = 64, alpha = 1e-4, float32-refined fine
    # path on the red-black resident kernel, multigrid COCG, 32-column slice FFTs) with a
    # shorter slice (J fine steps) so the oracle finishes in seconds
    w = W.get("c2_2d_n128").replace(J=J)
    log(f"parareal c2 shape n=128 N=64 J={J} M={M}")
    for it_gpu, it_or, e_or, e_ref, st, hg, ho in _parareal_case(
            ctx, w, M, "zero", dict(inner_rtol=1e-14, cgc_rtol=1e-14)):
        log(f"  iterations gpu {it_gpu} oracle {it_or}; vs oracle iterate {e_or:.2e}, vs serial fine {e_ref:.2e}")
        assert st == 0
        assert iterations_agree(it_gpu, it_or, ho, w.tol)
        assert e_ref < 1e-8
        assert e_or < 1e-8
        k = min(it_gpu, it_or)
        assert np.allclose(hg[:k], ho[:k], rtol=1e-4, atol=1e-13)


# ---------------------------------------------------------------- KL / gPC
def test_snapshot_kl_and_gpc_prediction(ctx):
    w = W.small_1d(n=15, N=4, J=4, d=3)
    n_t, p = 24, 2
    xi_t = W.draw_xi(n_t, w.d, 41)
    a_t = oracle_faces(w, xi_t)
    S = np.stack([prop.serial_fine(prop.Propagators(1, w.n, a_t[j], w.T, w.N, w.J, w.forcing),
                                   np.zeros(w.n), w.N).ravel() for j in range(n_t)])
    kl_o = snapshot.build(S, 1e-10)
    g_o = ogpc.fit(kl_o, S, xi_t, p)
    log(f"snapshot KL n_t={n_t} L={S.shape[1]} modes={kl_o.n_modes}")
    kl = ctx.kle_build(dev(S), 1e-10)
    lam_dbg = torch.empty(kl.n_modes, dtype=torch.float64, device="cuda")
    ctx.kle_export(kl, lam=lam_dbg)
    log(f"gpu lam {host(lam_dbg)}")
    log(f"orc lam {kl_o.lam}")
    assert kl.n_modes == kl_o.n_modes
    mean = torch.empty(S.shape[1], dtype=torch.float64, device="cuda")
    Wm = torch.empty((kl.n_modes, S.shape[1]), dtype=torch.float64, device="cuda")
    lam = torch.empty(kl.n_modes, dtype=torch.float64, device="cuda")
    ctx.kle_export(kl, mean, Wm, lam)
    assert rel(host(mean), kl_o.mean) < 1e-13
    assert np.allclose(host(lam), kl_o.lam, rtol=1e-9, atol=1e-12 * kl_o.lam[0])
    # basis rows agree up to sign on well-separated modes
    Wo = np.sqrt(kl_o.lam)[:, None] * kl_o.basis
    Wg = host(Wm)
    good = kl_o.lam > 1e-6 * kl_o.lam[0]
    for k in np.nonzero(good)[0]:
        sgn = np.sign(Wg[k] @ Wo[k])
        assert rel(sgn * Wg[k], Wo[k]) < 1e-7
    g = ctx.gpc_fit(kl, dev(xi_t), p)
    assert g.P == ogpc.n_terms(w.d, p)
    xi_e = W.draw_xi(6, w.d, 42)
    U0 = torch.empty((6, S.shape[1]), dtype=torch.float64, device="cuda")
    ctx.gpc_predict(g, dev(xi_e), U0)
    assert rel(host(U0), ogpc.predict(g_o, xi_e)) < 1e-10


def test_snapshot_gram_spectrum(ctx):
    # Gram matrix of random snapshots: all eigenvalues well separated from zero
    S = W.draw_normal((40, 333), 4)
    kl = ctx.kle_build(dev(S), 0.0)
    Sc = S - S.mean(0)
    want = np.sort(np.linalg.eigvalsh(Sc @ Sc.T / 40))[::-1][:kl.n_modes]
    lam = torch.empty(kl.n_modes, dtype=torch.float64, device="cuda")
    Wm = torch.empty((kl.n_modes, 333), dtype=torch.float64, device="cuda")
    ctx.kle_export(kl, W=Wm, lam=lam)
    got = host(lam)
    log(f"gram spectrum gpu {got[:5]} ... {got[-3:]}")
    log(f"gram spectrum np  {want[:5]} ... {want[-3:]}")
    assert kl.n_modes == 39
    assert np.allclose(got, want, rtol=1e-11)
    # rows of W are sqrt(lam_k) g_k: W W^T = diag(lam)
    Wh = host(Wm)
    assert np.allclose(Wh @ Wh.T, np.diag(want), atol=1e-11 * want[0])


def test_gpc_rejects_underdetermined(ctx):
    import paper_2510_26180_amd as K
    S = W.draw_normal((6, 20), 3)
    kl = ctx.kle_build(dev(S), 1e-12)
    with pytest.raises(K.KlecgcError) as e:
        ctx.gpc_fit(kl, dev(W.draw_xi(6, 4, 1)), 3)
    assert e.value.code == -4


# ---------------------------------------------------------------- errors and edges
def test_invalid_arguments_are_rejected(ctx):
    import paper_2510_26180_amd as K
    w = W.small_1d()
    a = dev(np.ones((1, w.n_faces)))
    x = torch.zeros((1, w.N, w.Nx), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    for bad in (dict(alpha=0.0), dict(alpha=1.0), dict(N=6), dict(J=0), dict(T=-1.0), dict(tol=0.0)):
        with pytest.raises(K.KlecgcError) as e:
            ctx.fine_propagate(spec_of(w, **bad), a, x, y)
        assert e.value.code == -1
    with pytest.raises(K.KlecgcError) as e:
        ctx.fine_propagate(spec_of(w, precision=1), a, x, y)
    assert e.value.code == -7


def test_nonfinite_sample_is_isolated(ctx):
    import paper_2510_26180_amd as K
    w = W.small_1d(n=15, N=4, J=4)
    M = 3
    xi = W.draw_xi(M, w.d, 5)
    a = oracle_faces(w, xi)
    a[1, 3] = np.nan
    U = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    iters, status, _, _ = ctx.parareal_solve(spec_of(w), dev(a), U, init=K.KC_INIT_ZERO)
    assert status[1] == K.KC_SAMPLE_NONFINITE
    assert status[0] == K.KC_SAMPLE_CONVERGED and status[2] == K.KC_SAMPLE_CONVERGED
    got = host(U)
    for m in (0, 2):
        P = prop.Propagators(1, w.n, a[m], w.T, w.N, w.J, w.forcing)
        assert rel(got[m], prop.serial_fine(P, np.zeros(w.n), w.N)) < 1e-8
