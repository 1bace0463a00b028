"""GPU parity of the initial-guess modes of parareal_solve (Algorithm 3 step 6, the learned
guess that replaces it, and the random guess of the Section 5 comparators), of the gPC-started
parareal at the 1D configuration end to end, and of two boundary options (the float32 copy of
the synthesised field, the active mask of fine_propagate), each against the CPU oracle.

Expected values come only from `oracle/`; inputs from `workloads`.  The GPU computes its own
training solutions, snapshot KL and gPC fit; the oracle computes its own.
"""
import numpy as np
import pytest

import workloads as W
from oracle import guess as oguess, gpc as ogpc, mlp as omlp, parareal as opar, prop, snapshot
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


# ---------------------------------------------------------------- random guess
@pytest.mark.parametrize("dim,n,N,J,seed", [(1, 31, 8, 8, 7), (1, 127, 16, 32, 2**63 + 5), (2, 12, 4, 4, 11),
                                            (2, 20, 8, 3, 0)])
def test_random_guess_first_iterate(ctx, dim, n, N, J, seed):
    # one iteration from the random guess: U^1 and the increment |U^1 - U^0| / |U^1| both
    # depend on every entry of U^0, which is drawn on the device from the counter stream
    import paper_2510_26180_amd as K
    log(f"random guess dim={dim} n={n} N={N} J={J} seed={seed}")
    w = (W.small_1d if dim == 1 else W.small_2d)(n=n, N=N, J=J)
    M = 3
    xi = W.draw_xi(M, w.d, 61)
    a = oracle_faces(w, xi)
    prob = spec_of(w, max_iter=1, inner_rtol=1e-14, cgc_rtol=1e-14)
    U = torch.empty((M, N, w.Nx), dtype=torch.float64, device="cuda")
    guess_out = np.zeros(M, np.int32)
    iters, status, hist, _ = ctx.parareal_solve(prob, dev(a), U, init=K.KC_INIT_RANDOM, seed=seed,
                                                guess_out=guess_out)
    U0 = oguess.random_guess(seed, M, N, w.Nx)
    got = host(U)
    assert (guess_out == K.KC_INIT_RANDOM).all()
    for m in range(M):
        P = prop.Propagators(dim, n, a[m], w.T, N, J, w.forcing)
        h = opar.parareal_diag(P, w.alpha, np.zeros(w.Nx), U0[m], w.tol, 1, keep=True)
        assert iters[m] == 1 and status[m] == K.KC_SAMPLE_MAXITER
        assert rel(got[m], h.iterates[1]) < 1e-10
        assert abs(hist[m, 0] - h.deltas[0]) <= 1e-10 * h.deltas[0]


def test_random_guess_parareal_c1(ctx):
    import paper_2510_26180_amd as K
    w = W.get("c1_1d_n127")
    M, seed = 4, 1234
    log(f"random-guess parareal c1 M={M}")
    xi = W.draw_xi(M, w.d, w.seed_eval)
    a = oracle_faces(w, xi)
    U = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    iters, status, hist, _ = ctx.parareal_solve(spec_of(w), dev(a), U, init=K.KC_INIT_RANDOM, seed=seed)
    U0 = oguess.random_guess(seed, M, w.N, w.Nx)
    got = host(U)
    for m in range(M):
        P = prop.Propagators(1, w.n, a[m], w.T, w.N, w.J, w.forcing)
        h = opar.parareal_diag(P, w.alpha, np.zeros(w.Nx), U0[m], w.tol, w.max_iter)
        ref = prop.serial_fine(P, np.zeros(w.Nx), w.N)
        log(f"  sample {m}: iterations gpu {iters[m]} oracle {h.iters}")
        assert status[m] == K.KC_SAMPLE_CONVERGED
        assert iterations_agree(int(iters[m]), h.iters, h.deltas, w.tol)
        if iters[m] == h.iters:
            assert rel(got[m], h.iterates[-1]) < 1e-10
        assert rel(got[m], ref) < 1e-8


# ---------------------------------------------------------------- gPC guess, c1 end to end
def test_gpc_parareal_c1(ctx):
    """Algorithm 3 at the 1D configuration: n_t = 50 training solutions, snapshot KL,
    Hermite gPC of total degree 3 (P = 35), then parareal from the gPC guess on the 8
    evaluation samples; the GPU and the oracle each compute their own training set."""
    import paper_2510_26180_amd as K
    w = W.get("c1_1d_n127")
    log(f"gPC parareal c1: n_t={w.n_train} p={w.gpc_degree} M={w.M}")
    prob = spec_of(w)
    fh = ctx.kle_build_field(w.dim, w.n, w.d, w.corr_len, w.sigma)
    xi_t = W.draw_xi(w.n_train, w.d, w.seed_train)
    xi_e = W.draw_xi(w.M, w.d, w.seed_eval)
    a_t = torch.empty((w.n_train, w.n_faces), dtype=torch.float64, device="cuda")
    a_e = torch.empty((w.M, w.n_faces), dtype=torch.float64, device="cuda")
    ctx.kle_synthesize(fh, dev(xi_t), a_t)
    ctx.kle_synthesize(fh, dev(xi_e), a_e)
    S = torch.empty((w.n_train, w.N, w.Nx), dtype=torch.float64, device="cuda")
    ctx.serial_fine_propagate(prob, a_t, None, S)
    kl = ctx.kle_build(S.view(w.n_train, -1), w.eps_kl)
    g = ctx.gpc_fit(kl, dev(xi_t), w.gpc_degree)
    U = torch.empty((w.M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    iters, status, hist, _ = ctx.parareal_solve(prob, a_e, U, init=K.KC_INIT_GPC, gpc=g, xi=dev(xi_e))
    got = host(U)
    # oracle
    at_o = oracle_faces(w, xi_t)
    ae_o = oracle_faces(w, xi_e)
    S_o = np.stack([prop.serial_fine(prop.Propagators(1, w.n, at_o[j], w.T, w.N, w.J, w.forcing),
                                     np.zeros(w.Nx), w.N).ravel() for j in range(w.n_train)])
    kl_o = snapshot.build(S_o, w.eps_kl)
    g_o = ogpc.fit(kl_o, S_o, xi_t, w.gpc_degree)
    assert g.P == ogpc.n_terms(w.d, w.gpc_degree) == 35
    U0 = ogpc.predict(g_o, xi_e).reshape(w.M, w.N, w.Nx)
    for m in range(w.M):
        P = prop.Propagators(1, w.n, ae_o[m], w.T, w.N, w.J, w.forcing)
        h = opar.parareal_diag(P, w.alpha, np.zeros(w.Nx), U0[m], w.tol, w.max_iter)
        ref = prop.serial_fine(P, np.zeros(w.Nx), w.N)
        log(f"  sample {m}: iterations gpu {iters[m]} oracle {h.iters}; error vs serial fine {rel(got[m], ref):.2e}")
        assert status[m] == K.KC_SAMPLE_CONVERGED
        assert iterations_agree(int(iters[m]), h.iters, h.deltas, w.tol)
        if iters[m] == h.iters:
            assert rel(got[m], h.iterates[-1]) < 1e-10
            assert np.allclose(hist[m, :iters[m]], h.deltas, rtol=1e-5, atol=1e-13)
        assert rel(got[m], ref) < 1e-8


# ---------------------------------------------------------------- learned guess
def _mlp_memorising(ctx, w, u_star_dev, nc):
    """A network whose weights are all zero, normalised on one row (the restriction of one
    solution): its output is 0, so the learned guess is the prolongation of that row."""
    O = w.N * nc * nc
    n_params = sum(int(np.prod(s)) for s in omlp.Params.shapes(w.d, 16, O))
    h = ctx.mlp_create(w.d, 16, O, params=torch.zeros(n_params, dtype=torch.float32, device="cuda"))
    Yc = torch.empty((1, O), dtype=torch.float32, device="cuda")
    ctx.grid_restrict(w.n, nc, u_star_dev, Yc)
    ctx.mlp_normalize_targets(h, Yc)
    return h


def test_mlp_init_equals_given_guess(ctx):
    # KC_INIT_MLP runs mlp_initial_guess inside parareal_solve: the same iterates as passing
    # that guess in (bitwise), and the serial fine solution of the oracle at the end
    import paper_2510_26180_amd as K
    w = W.small_2d(n=20, N=8, J=4, alpha=1e-2, d=6)
    M, nc, H = 3, 7, 32
    log(f"learned guess n={w.n} N={w.N} nc={nc}")
    O = w.N * nc * nc
    flat = W.draw_mlp_init(w.d, H, O, 71)
    h = ctx.mlp_create(w.d, H, O, params=dev(flat))
    Y = (W.draw_normal((5, O), 72, 0.02) + 0.02).astype(np.float32)
    ctx.mlp_normalize_targets(h, dev(Y))
    xi = W.draw_xi(M, w.d, 73)
    a = oracle_faces(w, xi)
    prob = spec_of(w, inner_rtol=1e-14, cgc_rtol=1e-14)
    U1 = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    g_out = np.zeros(M, np.int32)
    it1, st1, h1, _ = ctx.parareal_solve(prob, dev(a), U1, init=K.KC_INIT_MLP, mlp=h, xi=dev(xi), guess_out=g_out)
    G = torch.empty_like(U1)
    ctx.mlp_initial_guess(h, w.n, nc, w.N, dev(xi), G)
    U2 = torch.empty_like(U1)
    it2, st2, h2, _ = ctx.parareal_solve(prob, dev(a), U2, init=K.KC_INIT_GIVEN, init_U=G)
    assert (g_out == K.KC_INIT_MLP).all()
    assert np.array_equal(it1, it2) and np.array_equal(h1, h2)
    assert torch.equal(U1, U2)
    got = host(U1)
    for m in range(M):
        P = prop.Propagators(2, w.n, a[m], w.T, w.N, w.J, w.forcing)
        assert st1[m] == K.KC_SAMPLE_CONVERGED
        assert rel(got[m], prop.serial_fine(P, np.zeros(w.Nx), w.N)) < 1e-8


def _fallback_case(ctx, poison: bool):
    import paper_2510_26180_amd as K
    w = W.small_2d(n=12, N=4, J=4, alpha=1e-2, d=6)
    n_t, p, M = 40, 2, 8
    prob = spec_of(w, inner_rtol=1e-14, cgc_rtol=1e-14)
    xi_t = W.draw_xi(n_t, w.d, 51)
    xi_e = W.draw_xi(M, w.d, 52)
    # GPU: training solutions, snapshot KL, gPC; the memorised solution of evaluation sample 0
    fh = ctx.kle_build_field(2, w.n, w.d, w.corr_len, w.sigma)
    a_t = torch.empty((n_t, w.n_faces), dtype=torch.float64, device="cuda")
    a_e = torch.empty((M, w.n_faces), dtype=torch.float64, device="cuda")
    ctx.kle_synthesize(fh, dev(xi_t), a_t)
    ctx.kle_synthesize(fh, dev(xi_e), a_e)
    S = torch.empty((n_t, w.N, w.Nx), dtype=torch.float64, device="cuda")
    ctx.serial_fine_propagate(prob, a_t, None, S)
    g = ctx.gpc_fit(ctx.kle_build(S.view(n_t, -1), w.eps_kl), dev(xi_t), p)
    u_star = torch.empty((1, w.N, w.Nx), dtype=torch.float64, device="cuda")
    ctx.serial_fine_propagate(prob, a_e[:1].contiguous(), None, u_star)
    if poison:
        u_star[0, 1, 5] = float("nan")       # the learned guess turns NaN at one node of every sample
    h = _mlp_memorising(ctx, w, u_star, w.n)
    U = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    g_out = np.zeros(M, np.int32)
    iters, status, hist, _ = ctx.parareal_solve(prob, a_e, U, init=K.KC_INIT_MLP_GPC_FALLBACK, gpc=g, mlp=h,
                                                xi=dev(xi_e), guess_out=g_out)
    got = host(U)
    # oracle: its own training set, gPC and memorised solution; the same rule
    at_o = oracle_faces(w, xi_t)
    ae_o = oracle_faces(w, xi_e)
    S_o = np.stack([prop.serial_fine(prop.Propagators(2, w.n, at_o[j], w.T, w.N, w.J, w.forcing),
                                     np.zeros(w.Nx), w.N).ravel() for j in range(n_t)])
    g_o = ogpc.fit(snapshot.build(S_o, w.eps_kl), S_o, xi_t, p)
    Ug = ogpc.predict(g_o, xi_e).reshape(M, w.N, w.Nx)
    us_o = prop.serial_fine(prop.Propagators(2, w.n, ae_o[0], w.T, w.N, w.J, w.forcing), np.zeros(w.Nx), w.N)
    if poison:
        us_o[1, 5] = np.nan
    mu, _, _ = omlp.zscore(omlp.restrict(us_o, w.n, w.n).reshape(1, -1).astype(np.float32).astype(np.float64))
    learned = omlp.prolong(mu.reshape(w.N, w.Nx), w.n, w.n)
    out = []
    for m in range(M):
        P = prop.Propagators(2, w.n, ae_o[m], w.T, w.N, w.J, w.forcing)
        U0, use_f, dl, df = oguess.choose_guess(P, np.zeros(w.Nx), learned, Ug[m])
        h_o = opar.parareal_diag(P, w.alpha, np.zeros(w.Nx), U0, w.tol, w.max_iter)
        ref = prop.serial_fine(P, np.zeros(w.Nx), w.N)
        log(f"  sample {m}: defects learned {dl:.3e} gPC {df:.3e}: oracle keeps "
            f"{'gPC' if use_f else 'learned'}, gpu {'gPC' if g_out[m] == K.KC_INIT_GPC else 'learned'}; "
            f"iterations gpu {iters[m]} oracle {h_o.iters}")
        out.append((use_f, dl, df, int(g_out[m]), int(iters[m]), h_o, rel(got[m], ref), int(status[m])))
    return out


def test_mlp_gpc_fallback_rule(ctx):
    # evaluation sample 0 is the solution the network memorised (learned defect ~1e-8); for the
    # others the constant learned guess is worse than the gPC guess, and the rule moves them
    import paper_2510_26180_amd as K
    log("learned guess with gPC fallback")
    res = _fallback_case(ctx, poison=False)
    for use_f, dl, df, g_gpu, it_gpu, h_o, e_ref, st in res:
        assert g_gpu in (K.KC_INIT_MLP, K.KC_INIT_GPC)
        if abs(dl - df) > 1e-3 * max(dl, df):          # a decision not on a rounding edge
            assert (g_gpu == K.KC_INIT_GPC) == use_f
            assert iterations_agree(it_gpu, h_o.iters, h_o.deltas, 1e-8)
        assert st == K.KC_SAMPLE_CONVERGED and e_ref < 1e-8
    assert res[0][3] == K.KC_INIT_MLP
    assert sum(r[3] == K.KC_INIT_GPC for r in res) >= 5


def test_mlp_gpc_fallback_from_non_finite_learned_guess(ctx):
    import paper_2510_26180_amd as K
    log("learned guess with a NaN entry: every sample falls back to gPC")
    res = _fallback_case(ctx, poison=True)
    for use_f, dl, df, g_gpu, it_gpu, h_o, e_ref, st in res:
        assert np.isnan(dl) and use_f
        assert g_gpu == K.KC_INIT_GPC
        assert iterations_agree(it_gpu, h_o.iters, h_o.deltas, 1e-8)
        assert st == K.KC_SAMPLE_CONVERGED and e_ref < 1e-8


def test_guess_modes_reject_missing_handles(ctx):
    import paper_2510_26180_amd as K
    w = W.small_2d(n=8, N=4, J=2)
    a = dev(oracle_faces(w, W.draw_xi(1, w.d, 3)))
    U = torch.empty((1, w.N, w.Nx), dtype=torch.float64, device="cuda")
    for init in (K.KC_INIT_MLP, K.KC_INIT_MLP_GPC_FALLBACK, K.KC_INIT_GPC):
        with pytest.raises(K.KlecgcError) as e:
            ctx.parareal_solve(spec_of(w), a, U, init=init, xi=dev(np.zeros((1, w.d))))
        assert e.value.code == -1
    h = ctx.mlp_create(w.d, 8, 3 * w.N * 4)            # n_out / N = 12 is not a square
    with pytest.raises(K.KlecgcError) as e:
        ctx.parareal_solve(spec_of(w), a, U, init=K.KC_INIT_MLP, mlp=h, xi=dev(np.zeros((1, w.d))))
    assert e.value.code == -1


# ---------------------------------------------------------------- boundary options
@pytest.mark.parametrize("w", [W.get("c1_1d_n127"), W.small_2d(n=37, d=10)])
def test_field_synthesis_float32_copy(ctx, w):
    log(f"field synthesis with float32 copy dim={w.dim} n={w.n}")
    M = 4
    xi = W.draw_xi(M, w.d, 81)
    want = oracle_faces(w, xi)
    fh = ctx.kle_build_field(w.dim, w.n, w.d, w.corr_len, w.sigma)
    a = torch.empty((M, w.n_faces), dtype=torch.float64, device="cuda")
    a32 = torch.empty((M, w.n_faces), dtype=torch.float32, device="cuda")
    ctx.kle_synthesize(fh, dev(xi), a, a32)
    assert torch.equal(a32, a.to(torch.float32))
    assert rel(host(a), want) < 1e-12
    assert np.abs(host(a32).astype(np.float64) - want).max() <= (2.0 ** -24 + 1e-11) * np.abs(want).max()


@pytest.mark.parametrize("dim,n,prec", [(1, 31, 0), (2, 20, 0), (2, 72, 1), (2, 150, 1)])
def test_fine_propagate_active_mask(ctx, dim, n, prec):
    log(f"fine propagate with an active mask dim={dim} n={n} prec={prec}")
    w = (W.small_1d if dim == 1 else W.small_2d)(n=n, N=4, J=3)
    M = 5
    xi = W.draw_xi(M, w.d, 91)
    a = oracle_faces(w, xi)
    starts = W.draw_uniform((M, w.N, w.Nx), 92) * 0.05
    mask = np.array([1, 0, 1, 1, 0], np.uint8)
    end = torch.full((M, w.N, w.Nx), -7.0, dtype=torch.float64, device="cuda")
    ctx.fine_propagate(spec_of(w, precision=prec, inner_rtol=1e-14), dev(a), dev(starts), end,
                       active=dev(mask))
    got = host(end)
    for m in range(M):
        if not mask[m]:
            assert (got[m] == -7.0).all()
            continue
        P = prop.Propagators(dim, n, a[m], w.T, w.N, w.J, w.forcing)
        for s in range(w.N):
            assert rel(got[m, s], P.F(starts[m, s])) < 1e-11


# ---------------------------------------------------------------- Algorithm 1 and the alpha sweep
@pytest.mark.parametrize("dim,n,N,J,init", [(1, 31, 8, 8, "zero"), (1, 127, 16, 32, "random"), (2, 12, 4, 4, "zero"),
                                            (2, 20, 8, 3, "random")])
def test_sequential_cgc_iterates(ctx, dim, n, N, J, init):
    """Algorithm 1 (sequential CGC) for exactly K iterations against the oracle's iterates,
    K = 1, 2 and N; at K = N the iterate is the serial fine solution (finite termination)."""
    import paper_2510_26180_amd as K_
    w = (W.small_1d if dim == 1 else W.small_2d)(n=n, N=N, J=J)
    M, seed = 2, 77
    xi = W.draw_xi(M, w.d, 63)
    a = oracle_faces(w, xi)
    mode = K_.KC_INIT_ZERO if init == "zero" else K_.KC_INIT_RANDOM
    U0 = np.zeros((M, N, w.Nx)) if init == "zero" else oguess.random_guess(seed, M, N, w.Nx)
    ref = [opar.parareal_sequential(prop.Propagators(dim, n, a[m], w.T, N, J, w.forcing), np.zeros(w.Nx), U0[m], N)
           for m in range(M)]
    for Kit in (1, 2, N):
        log(f"sequential CGC dim={dim} n={n} N={N} J={J} init={init} K={Kit}")
        prob = spec_of(w, max_iter=Kit, tol=1e-300, inner_rtol=1e-14)
        U = torch.empty((M, N, w.Nx), dtype=torch.float64, device="cuda")
        iters, status, hist, _ = ctx.parareal_solve_sequential(prob, dev(a), U, init=mode, seed=seed)
        got = host(U)
        for m in range(M):
            assert iters[m] == Kit
            assert rel(got[m], ref[m][Kit]) < 1e-11
            # both iterates agree with the oracle's to ~1e-12 relative, so their increment to ~1e-11
            inc = opar.increment(ref[m][Kit], ref[m][Kit - 1])
            assert abs(hist[m, Kit - 1] - inc) <= 1e-10
        if Kit == N:
            for m in range(M):
                P = prop.Propagators(dim, n, a[m], w.T, N, J, w.forcing)
                assert rel(got[m], prop.serial_fine(P, np.zeros(w.Nx), N)) < 1e-12


def test_alpha_sweep_c1(ctx):
    """The twist parameter at the 1D configuration: for alpha = 1e-1, 1e-2, 1e-4 the
    diagonalised CGC (Algorithm 2) stops after the oracle's iteration count; Algorithm 1
    (alpha = 0, sequential CGC) likewise.  Smaller alpha moves Algorithm 2 towards
    Algorithm 1's convergence."""
    import paper_2510_26180_amd as K_
    w = W.get("c1_1d_n127")
    M = 4
    xi = W.draw_xi(M, w.d, w.seed_eval)
    a = oracle_faces(w, xi)
    counts = {}
    for alpha in (1e-1, 1e-2, 1e-4):
        log(f"alpha sweep c1: alpha={alpha}")
        U = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
        its, st, _, _ = ctx.parareal_solve(spec_of(w, alpha=alpha), dev(a), U, init=K_.KC_INIT_ZERO)
        want = []
        for m in range(M):
            P = prop.Propagators(1, w.n, a[m], w.T, w.N, w.J, w.forcing)
            h = opar.parareal_diag(P, alpha, np.zeros(w.Nx), np.zeros((w.N, w.Nx)), w.tol, w.max_iter)
            want.append(h.iters)
            assert iterations_agree(int(its[m]), h.iters, h.deltas, w.tol)
        counts[alpha] = (its.tolist(), want)
    U = torch.empty((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    its, st, hist, _ = ctx.parareal_solve_sequential(spec_of(w), dev(a), U, init=K_.KC_INIT_ZERO)
    for m in range(M):
        P = prop.Propagators(1, w.n, a[m], w.T, w.N, w.J, w.forcing)
        seq = opar.parareal_sequential(P, np.zeros(w.Nx), np.zeros((w.N, w.Nx)), w.N)
        deltas = [opar.increment(seq[k], seq[k - 1]) for k in range(1, w.N + 1)]
        k_or = next(k for k, d in enumerate(deltas, 1) if d <= w.tol)
        assert iterations_agree(int(its[m]), k_or, deltas, w.tol)
    counts[0.0] = its.tolist()
    log(f"  iterations by alpha (gpu, oracle): {counts}")
