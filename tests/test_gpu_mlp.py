"""GPU parity of the learned initial guess (BF16 MFMA MLP, grid transfer) against the
oracle's FP64 MLP with the kernels' bfloat16 rounding points mirrored.

Tolerances.  Both sides round the same GEMM operands to bfloat16, but the kernel
computes the pre-rounding values in FP32 and the oracle in FP64, so an operand that
lies within ~1e-7 relative of a rounding boundary can land one bfloat16 ulp (2^-8
relative) apart.  Emulating the kernel's FP32 arithmetic on the CPU gives at most a
few 1e-4 (max-norm relative) from such flips at these sizes and ~1e-7 everywhere
else, so the tests bound the max error by a few flips (2e-3 forward, 5e-3 gradients)
and require almost every element to agree to FP32 accumulation accuracy.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mlp as omlp
from tests.gpu_helpers import dev, host, log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(10, 96, 200, 70), (10, 256, 1064, 300), (3, 64, 64, 1)]


@pytest.fixture(scope="module")
def ctx():
    import paper_2510_26180_amd as K
    c = K.Context(0)
    yield c
    c.close()


def _net(ctx, n_in, H, O, seed=5, bias=0.1):
    flat = W.draw_mlp_init(n_in, H, O, seed)
    L = omlp.Params.shapes(n_in, H, O)
    o = 0
    for s in L:                       # non-zero biases so that the bias paths are exercised
        k = int(np.prod(s))
        if len(s) == 1:
            flat[o:o + k] = bias * np.cos(np.arange(k))
        o += k
    h = ctx.mlp_create(n_in, H, O, params=dev(flat))
    assert h.n_params == flat.size
    return h, omlp.Params.from_flat(flat.astype(np.float64), n_in, H, O), flat


def _agree(got, want, max_tol, frac_tol, small):
    e = np.abs(got - want)
    m = max(np.abs(want).max(), 1e-300)
    frac = float((e > small * m).mean())
    return float(e.max() / m), frac


@pytest.mark.parametrize("shape", SHAPES)
def test_mlp_forward(ctx, shape):
    n_in, H, O, B = shape
    log(f"mlp forward n_in={n_in} H={H} O={O} B={B}")
    h, p, _ = _net(ctx, n_in, H, O)
    X = W.draw_xi(B, n_in, 6)
    Y = torch.empty((B, O), dtype=torch.float32, device="cuda")
    ctx.mlp_predict(h, dev(X), Y)
    want, _ = omlp.forward(p, X, mirror_bf16=True)
    mx, frac = _agree(host(Y).astype(np.float64), want, 2e-3, 0.02, 1e-5)
    log(f"  max rel {mx:.2e}, fraction beyond 1e-5: {frac:.4f}")
    assert mx <= 2e-3 and frac <= 0.02


@pytest.mark.parametrize("shape", SHAPES[:2])
def test_mlp_gradients(ctx, shape):
    n_in, H, O, B = shape
    log(f"mlp gradients n_in={n_in} H={H} O={O} B={B}")
    h, p, _ = _net(ctx, n_in, H, O)
    X = W.draw_xi(B, n_in, 6)
    T = W.draw_normal((B, O), 7).astype(np.float32)
    g = torch.empty(h.n_params, dtype=torch.float32, device="cuda")
    loss = ctx.mlp_grad(h, dev(X), dev(T), g)
    wl, wg = omlp.loss_and_grad(p, X, T.astype(np.float64), mirror_bf16=True)
    assert abs(loss - wl) <= 1e-5 * wl
    got = omlp.Params.from_flat(host(g), n_in, H, O)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        mx, frac = _agree(getattr(got, k), wg[k], 5e-3, 0.1, 1e-4)
        log(f"  {k}: max rel {mx:.2e}, fraction beyond 1e-4: {frac:.4f}")
        assert mx <= 5e-3 and frac <= 0.1, k


def test_mlp_first_adam_step(ctx):
    n_in, H, O, B = 10, 96, 200, 70
    h, p, flat = _net(ctx, n_in, H, O)
    X = W.draw_xi(B, n_in, 8)
    T = W.draw_normal((B, O), 9).astype(np.float32)
    lr = 1e-3
    losses = ctx.mlp_train(h, dev(X), dev(T), epochs=1, batch=B, lr=lr)
    after = torch.empty(h.n_params, dtype=torch.float32, device="cuda")
    ctx.mlp_get_params(h, params=after)
    step_gpu = host(after).astype(np.float64) - flat.astype(np.float64)
    wl, wg = omlp.loss_and_grad(p, X, T.astype(np.float64), mirror_bf16=True)
    m = {k: np.zeros_like(v) for k, v in wg.items()}
    v = {k: np.zeros_like(x) for k, x in wg.items()}
    before = omlp.Params.from_flat(flat.astype(np.float64), n_in, H, O)
    omlp.adam_step(p, wg, m, v, 1, lr)
    step_or = p.flat() - before.flat()
    d = np.abs(step_gpu - step_or)
    log(f"  loss {losses[0]:.6e} vs {wl:.6e}; step diff max {d.max():.2e}, frac>1e-3 lr {(d > 1e-3 * lr).mean():.4f}")
    assert abs(losses[0] - wl) <= 1e-5 * wl
    assert d.max() <= 2.0 * lr * (1 + 1e-3)          # a step is at most lr in size
    assert (d > 1e-3 * lr).mean() <= 0.01


def test_mlp_training_tracks_oracle_and_decreases(ctx):
    n_in, H, O, n = 4, 64, 96, 200
    h, p, flat = _net(ctx, n_in, H, O, seed=11, bias=0.0)
    X = W.draw_xi(n, n_in, 12)
    # a smooth learnable target: a fixed random function of xi, then z-scored
    A = W.draw_normal((n_in, O), 13, 0.7)
    Traw = np.sin(X @ A).astype(np.float32)
    Tdev = dev(Traw)
    ctx.mlp_normalize_targets(h, Tdev)
    mu, sd, Tz = omlp.zscore(Traw.astype(np.float64))
    assert rel(host(Tdev), Tz) <= 1e-6
    epochs, batch, lr, lr_final = 3, 64, 3e-3, 1e-3
    perm = W.draw_perms(epochs, n, 14)
    losses = ctx.mlp_train(h, dev(X), Tdev, epochs=epochs, batch=batch, lr=lr, perm=dev(perm), lr_final=lr_final)
    # oracle: same permutations, same mini-batches (the last one ragged), FP64 masters
    m = {k: 0.0 for k in ("W1", "b1", "W2", "b2", "W3", "b3")}
    v = dict(m)
    t = 0
    want = []
    for ep in range(epochs):
        lr_ep = lr * (lr_final / lr) ** (ep / (epochs - 1))      # geometric decay per epoch
        tot = 0.0
        for off in range(0, n, batch):
            rows = perm[ep, off:off + batch]
            l, g = omlp.loss_and_grad(p, X[rows], Tz[rows], mirror_bf16=True)
            tot += l * len(rows)
            t += 1
            omlp.adam_step(p, g, m, v, t, lr_ep)
        want.append(tot / n)
    log(f"  losses gpu {losses} oracle {np.array(want)}")
    assert np.allclose(losses, want, rtol=2e-3)
    after = torch.empty(h.n_params, dtype=torch.float32, device="cuda")
    ctx.mlp_get_params(h, params=after)
    d = np.abs(host(after).astype(np.float64) - p.flat())
    log(f"  params after {epochs * 4} steps: max diff {d.max():.2e}, frac>1e-2 lr {(d > 1e-2 * lr).mean():.4f}")
    assert (d > 1e-2 * lr).mean() <= 0.02
    longer = ctx.mlp_train(h, dev(X), Tdev, epochs=40, batch=batch, lr=lr)
    assert longer[-1] < 0.5 * losses[0]


def test_normalize_targets(ctx):
    O = 300
    Y = W.draw_normal((33, O), 15, 2.0).astype(np.float32) + 5.0
    Y[:, 7] = 3.0                                           # constant column: std -> 1
    h = ctx.mlp_create(2, 8, O)
    Yd = dev(Y)
    ctx.mlp_normalize_targets(h, Yd)
    mu, sd, Z = omlp.zscore(Y.astype(np.float64))
    mean = torch.empty(O, dtype=torch.float32, device="cuda")
    std = torch.empty(O, dtype=torch.float32, device="cuda")
    ctx.mlp_get_params(h, mean=mean, std=std)
    assert rel(host(mean), mu) <= 1e-6 and rel(host(std), sd) <= 1e-6
    assert np.abs(host(Yd) - Z).max() <= 1e-5
    assert host(std)[7] == 1.0


@pytest.mark.parametrize("n,nc", [(20, 7), (15, 7), (33, 32), (128, 32), (1, 3)])
def test_grid_restrict(ctx, n, nc):
    R = 5
    U = W.draw_normal((R, n * n), 16)
    Yc = torch.empty((R, nc * nc), dtype=torch.float32, device="cuda")
    ctx.grid_restrict(n, nc, dev(U), Yc)
    want = omlp.restrict(U, n, nc)
    assert np.abs(host(Yc) - want).max() <= 1e-6 * max(np.abs(want).max(), 1.0)


@pytest.mark.parametrize("n,nc,N", [(20, 7, 4), (128, 32, 3), (9, 12, 2)])
def test_mlp_initial_guess_prolongs_denormalised_output(ctx, n, nc, N):
    # W3 = 0, so the network output is exactly b3: the test isolates de-normalisation
    # and prolongation (FP64) from the BF16 GEMMs.
    n_in, H = 5, 32
    O = N * nc * nc
    flat = W.draw_mlp_init(n_in, H, O, 17)
    L = omlp.Params.shapes(n_in, H, O)
    oW3 = sum(int(np.prod(s)) for s in L[:4])
    flat[oW3:oW3 + H * O] = 0.0
    b3 = W.draw_normal(O, 18).astype(np.float32)
    flat[oW3 + H * O:] = b3
    h = ctx.mlp_create(n_in, H, O, params=dev(flat))
    Y = (W.draw_normal((12, O), 19, 3.0) + 1.0).astype(np.float32)
    ctx.mlp_normalize_targets(h, dev(Y))
    mean = torch.empty(O, dtype=torch.float32, device="cuda")
    std = torch.empty(O, dtype=torch.float32, device="cuda")
    ctx.mlp_get_params(h, mean=mean, std=std)
    M = 3
    xi = W.draw_xi(M, n_in, 20)
    U0 = torch.empty((M, N, n * n), dtype=torch.float64, device="cuda")
    ctx.mlp_initial_guess(h, n, nc, N, dev(xi), U0)
    mu, sd, _ = omlp.zscore(Y.astype(np.float64))
    coarse = (mu + sd * b3.astype(np.float64)).reshape(N, nc * nc)
    want = omlp.prolong(coarse, nc, n)
    for m in range(M):
        assert rel(host(U0)[m], want) <= 1e-6


def test_mlp_rejects_bad_arguments(ctx):
    import paper_2510_26180_amd as K
    h = ctx.mlp_create(3, 16, 40)
    U0 = torch.empty((1, 4, 25), dtype=torch.float64, device="cuda")
    with pytest.raises(K.KlecgcError) as e:
        ctx.mlp_initial_guess(h, 5, 3, 4, dev(np.zeros((1, 3))), U0)    # 4 * 3^2 != 40
    assert e.value.code == -1
    with pytest.raises(K.KlecgcError) as e:
        ctx.mlp_create(0, 16, 40)
    assert e.value.code == -1
    with pytest.raises(K.KlecgcError) as e:
        ctx.mlp_train(h, dev(np.zeros((2, 3))), dev(np.zeros((2, 40), np.float32)), 1, 0, 1e-3)
    assert e.value.code == -1


def test_trained_network_gains_over_no_guess(ctx):
    """Train the MLP on serial-fine solutions of a small 2D problem, then solve fresh
    samples from (a) the zero guess, (b) the gPC guess, (c) the MLP guess.  The network
    must cut the iteration count against (a) and every run must reach the oracle's
    serial fine solution to 1e-8; the comparison with (b) is reported."""
    import paper_2510_26180_amd as K
    from oracle import prop
    from tests.gpu_helpers import oracle_faces
    w = W.small_2d(n=20, N=8, J=8, alpha=1e-2, d=6, M=32)
    prob = K.ProblemSpec.from_workload(w)
    n_t, nc, H = 512, 9, 64
    fh = ctx.kle_build_field(w.dim, w.n, w.d, w.corr_len, w.sigma)
    xi_t = dev(W.draw_xi(n_t, w.d, 31))
    xi_e_np = W.draw_xi(w.M, w.d, 32)
    xi_e = dev(xi_e_np)
    a_t = torch.empty((n_t, w.n_faces), dtype=torch.float64, device="cuda")
    a_e = torch.empty((w.M, w.n_faces), dtype=torch.float64, device="cuda")
    ctx.kle_synthesize(fh, xi_t, a_t)
    ctx.kle_synthesize(fh, xi_e, a_e)
    S = torch.empty((n_t, w.N, w.Nx), dtype=torch.float64, device="cuda")
    ctx.serial_fine_propagate(prob, a_t, None, S)
    O = w.N * nc * nc
    Yc = torch.empty((n_t, O), dtype=torch.float32, device="cuda")
    ctx.grid_restrict(w.n, nc, S, Yc)
    h = ctx.mlp_create(w.d, H, O, params=dev(W.draw_mlp_init(w.d, H, O, 33)))
    ctx.mlp_normalize_targets(h, Yc)
    epochs = 300
    losses = ctx.mlp_train(h, xi_t, Yc, epochs=epochs, batch=64, lr=1e-3, lr_final=1e-5,
                           perm=dev(W.draw_perms(epochs, n_t, 34)))
    kl = ctx.kle_build(S.view(n_t, -1), w.eps_kl)
    gpc = ctx.gpc_fit(kl, xi_t, 2)
    U = torch.empty((w.M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    its = {}
    its["zero"], st0, _, _ = ctx.parareal_solve(prob, a_e, U, init=K.KC_INIT_ZERO)
    its["gpc"], st1, _, _ = ctx.parareal_solve(prob, a_e, U, init=K.KC_INIT_GPC, gpc=gpc, xi=xi_e)
    ctx.mlp_initial_guess(h, w.n, nc, w.N, xi_e, U)
    its["mlp"], st2, _, _ = ctx.parareal_solve(prob, a_e, U, init=K.KC_INIT_GIVEN, init_U=U)
    log(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}; mean iterations " +
        ", ".join(f"{k} {v.mean():.2f}" for k, v in its.items()))
    assert all((s == K.KC_SAMPLE_CONVERGED).all() for s in (st0, st1, st2))
    assert its["mlp"].mean() < its["zero"].mean() - 1.0
    a0 = oracle_faces(w, xi_e_np[:1])[0]
    ref = prop.serial_fine(prop.Propagators(w.dim, w.n, a0, w.T, w.N, w.J, w.forcing), np.zeros(w.Nx), w.N)
    assert rel(host(U)[0], ref) <= 1e-8
