"""GPU parity of the nonlinear models (Burgers, Section 5.2; Allen-Cahn, Section 5.3) and of the
Newton coarse grid correction with the averaged Jacobian (Section 3.2, eq. Newton2) against
oracle/nonlinear.py, through the C ABI: F slice by slice, the sequential G and F sweeps, one
Newton-CGC (iterate and Newton step count), Algorithm 2 from the zero and random guesses
(iteration counts, iterates, error history), Algorithm 1 to finite termination, the discrete
Allen-Cahn energy along the GPU serial fine solution, and both Section 5 configurations on two
samples for a few iterations.
"""
import numpy as np
import pytest

import paper_2510_26180_amd as K
import workloads as W
from oracle import guess as oguess, nonlinear as onl
from tests.gpu_helpers import dev, host, log, rel

pytestmark = pytest.mark.gpu

MODELS = {"burgers": K.KC_MODEL_BURGERS, "allen_cahn": K.KC_MODEL_ALLEN_CAHN}
EPS = {"burgers": (1.0, 3.0), "allen_cahn": (0.2, 0.9)}


@pytest.fixture(scope="module")
def ctx():
    c = K.Context(0)
    yield c
    c.close()


def _spec(model, n, N, J, T=1.0, alpha=0.1, tol=0.0, max_iter=30):
    return K.ModelSpec(MODELS[model], n, T, N, J, alpha, tol=tol, max_iter=max_iter, newton_tol=1e-13,
                       newton_max_iter=60)


def _eps(model, M, seed):
    lo, hi = EPS[model]
    return lo + (hi - lo) * W.draw_uniform((M,), seed)


def _props(ms, e):
    return onl.NLPropagators(ms.model, ms.n, e, ms.T, ms.N, ms.J, 1e-13, 60)


@pytest.mark.parametrize("model", ["burgers", "allen_cahn"])
@pytest.mark.parametrize("n", [13, 70])
def test_fine_propagate_matches_oracle(ctx, model, n):
    ms = _spec(model, n, 4, 5)
    M = 2
    e = _eps(model, M, 3)
    base = onl.MODELS[ms.model](n, 1.0).initial_value()
    start = base[None, None, :] * (0.5 + W.draw_uniform((M, 4, 1), 4)) + 0.05 * (W.draw_uniform((M, 4, n), 5) - 0.5)
    end = dev(np.zeros_like(start))
    log(f"nl fine {model} n={n}")
    ctx.model_fine_propagate(ms, dev(e), dev(start), end)
    got = host(end)
    for m in range(M):
        P = _props(ms, e[m])
        for s in range(4):
            assert rel(got[m, s], P.F(start[m, s])) < 1e-12


@pytest.mark.parametrize("model", ["burgers", "allen_cahn"])
def test_coarse_and_serial_sweeps_match_oracle(ctx, model):
    ms = _spec(model, 31, 6, 4)
    M = 2
    e = _eps(model, M, 6)
    Uc = dev(np.zeros((M, 6, 31)))
    Uf = dev(np.zeros((M, 6, 31)))
    ctx.model_coarse_propagate(ms, dev(e), Uc)
    ctx.model_serial_fine(ms, dev(e), Uf)
    gc, gf = host(Uc), host(Uf)
    for m in range(M):
        P = _props(ms, e[m])
        u0 = P.prob.initial_value()
        assert rel(gc[m], onl.coarse_sweep(P, u0)) < 1e-12
        assert rel(gf[m], onl.serial_fine(P, u0)) < 1e-12


@pytest.mark.parametrize("model", ["burgers", "allen_cahn"])
def test_newton_cgc_matches_oracle(ctx, model):
    n, N = 21, 6
    ms = _spec(model, n, N, 3)
    M = 2
    e = _eps(model, M, 8)
    base = onl.MODELS[ms.model](n, 1.0).initial_value()
    Uk = np.tile(base, (M, N, 1)) * (0.8 + 0.2 * W.draw_uniform((M, N, 1), 9))
    Fv = Uk + 0.01 * (W.draw_uniform((M, N, n), 10) - 0.5)
    Unew = dev(np.zeros_like(Uk))
    its = ctx.model_cgc_solve(ms, dev(e), dev(Uk), dev(Fv), Unew)
    got = host(Unew)
    for m in range(M):
        P = _props(ms, e[m])
        b = onl.cgc_b(P, ms.alpha, Uk[m], Fv[m])
        want, oits = onl.newton_cgc(P, ms.alpha, Uk[m], b)
        assert abs(int(its[m]) - oits) <= 1, (its[m], oits)
        assert rel(got[m], want) < 1e-11, rel(got[m], want)
        assert np.abs(onl.all_at_once_residual(P, ms.alpha, got[m], b)).max() < 1e-10


@pytest.mark.parametrize("model", ["burgers", "allen_cahn"])
@pytest.mark.parametrize("init", ["zero", "random"])
def test_alg2_matches_oracle(ctx, model, init):
    n, N, J = 23, 6, 4
    ms = _spec(model, n, N, J, tol=1e-10, max_iter=40)
    M = 2
    e = _eps(model, M, 12)
    Uref = dev(np.zeros((M, N, n)))
    ctx.model_serial_fine(ms, dev(e), Uref)
    U = dev(np.zeros((M, N, n)))
    mode = K.KC_INIT_ZERO if init == "zero" else K.KC_INIT_RANDOM
    iters, status, hist, errs = ctx.model_parareal_solve(ms, dev(e), U, init=mode, seed=21, ref=Uref)
    got, ref = host(U), host(Uref)
    for m in range(M):
        P = _props(ms, e[m])
        u0 = P.prob.initial_value()
        oref = onl.serial_fine(P, u0)
        assert rel(ref[m], oref) < 1e-12
        U0 = np.zeros((N, n)) if init == "zero" else oguess.uniform_counter(21, m * N * n, N * n).reshape(N, n)
        h = onl.parareal_diag(P, ms.alpha, u0, U0, ms.tol, ms.max_iter, oref)
        assert status[m] == K.KC_SAMPLE_CONVERGED
        if abs(h.deltas[-1] - ms.tol) > 0.01 * ms.tol:
            assert iters[m] == h.iters, (iters[m], h.iters)
        assert rel(got[m], h.U) < 1e-10
        k = min(int(iters[m]), h.iters)
        assert np.abs(errs[m, :k + 1] - np.array(h.errors[:k + 1])).max() < 1e-9 * np.abs(oref).max()


@pytest.mark.parametrize("model", ["burgers", "allen_cahn"])
def test_alg1_finite_termination(ctx, model):
    n, N, J = 17, 5, 3
    ms = _spec(model, n, N, J, tol=0.0, max_iter=N)
    M = 2
    e = _eps(model, M, 14)
    Uref = dev(np.zeros((M, N, n)))
    ctx.model_serial_fine(ms, dev(e), Uref)
    U = dev(np.zeros((M, N, n)))
    iters, status, hist, errs = ctx.model_parareal_solve(ms, dev(e), U, init=K.KC_INIT_ZERO, ref=Uref,
                                                         sequential=True)
    got, ref = host(U), host(Uref)
    for m in range(M):
        scale = np.abs(ref[m]).max()
        for k in range(1, N + 1):
            assert errs[m, k, :k].max() < 1e-12 * scale
        P = _props(ms, e[m])
        h = onl.parareal_sequential(P, P.prob.initial_value(), np.zeros((N, n)), 0.0, N)
        assert rel(got[m], h.U) < 1e-12


def test_allen_cahn_energy_decays_on_gpu(ctx):
    n, N, J = 63, 12, 8
    ms = _spec("allen_cahn", n, N, J, T=6.0)
    e = np.array([0.1, 0.5])
    U = dev(np.zeros((2, N, n)))
    ctx.model_serial_fine(ms, dev(e), U)
    got = host(U)
    for m in range(2):
        prob = onl.AllenCahn(n, e[m])
        E = [prob.energy(prob.initial_value())] + [prob.energy(u) for u in got[m]]
        assert all(E[i + 1] <= E[i] + 1e-13 for i in range(N))


@pytest.mark.parametrize("name", ["f1_burgers_s52", "f1_allen_cahn_s53"])
def test_section_5_configuration_on_two_samples(ctx, name):
    w = W.MODELS[name]
    ms = K.ModelSpec(w.model, w.n, w.T, w.N, w.J, w.alpha, tol=0.0, max_iter=2)
    M = 2
    _, c, _ = W.draw_model_params(w, M, 61)
    Uref = dev(np.zeros((M, w.N, w.n)))
    ctx.model_serial_fine(ms, dev(c), Uref)
    U = dev(np.zeros((M, w.N, w.n)))
    log(f"{name}: 2 iterations from the random guess")
    iters, status, hist, errs = ctx.model_parareal_solve(ms, dev(c), U, init=K.KC_INIT_RANDOM, seed=3, ref=Uref)
    got, ref = host(U), host(Uref)
    for m in range(M):
        P = onl.NLPropagators(w.model, w.n, c[m], w.T, w.N, w.J)
        u0 = P.prob.initial_value()
        oref = onl.serial_fine(P, u0)
        assert rel(ref[m], oref) < 1e-11
        U0 = oguess.uniform_counter(3, m * w.N * w.n, w.N * w.n).reshape(w.N, w.n)
        h = onl.parareal_diag(P, w.alpha, u0, U0, 0.0, 2, oref)
        assert rel(got[m], h.U) < 1e-9, rel(got[m], h.U)
