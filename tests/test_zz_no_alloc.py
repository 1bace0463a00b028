"""The allocation-free fine propagator (fine_propagate_noalloc) against fine_propagate.

Both run the same kernels on the same inputs, so their outputs must agree bit for bit;
both are also checked against the oracle's F at the float64 bar.  Two calls in a row share
the device scratch array, the second one smaller than the first, so stale contents of the
first call must not leak into the second.  A call whose workspace exceeds the array is
rejected before it writes any output.
"""
import numpy as np
import pytest

import workloads as W
from oracle import prop
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


def _case(ctx, w, M, prec, seed, active=None):
    xi = W.draw_xi(M, w.d, seed)
    a = oracle_faces(w, xi)
    starts = W.draw_uniform((M, w.N, w.Nx), seed + 1) * 0.05
    prob = spec_of(w, precision=prec, inner_rtol=1e-14)
    want = torch.full((M, w.N, w.Nx), -3.0, dtype=torch.float64, device="cuda")
    got = torch.full_like(want, -3.0)
    act = None if active is None else dev(np.asarray(active, np.uint8))
    ctx.fine_propagate(prob, dev(a), dev(starts), want, active=act)
    ctx.fine_propagate_noalloc(prob, dev(a), dev(starts), got, active=act)
    return a, starts, want, got


@pytest.mark.parametrize("first,second", [
    # (dim, n, N, J, M, precision) of two calls in a row, the second smaller
    ((2, 72, 4, 4, 3, 1), (2, 40, 2, 3, 1, 1)),       # red-black resident, then full-system resident
    ((2, 150, 2, 2, 1, 1), (2, 130, 2, 2, 1, 1)),     # multigrid (chunks of what the array holds)
    ((2, 20, 4, 3, 2, 0), (1, 31, 4, 5, 2, 0)),       # float64 PCG, then 1D Thomas
])
def test_noalloc_matches_fine_propagate(ctx, first, second):
    for dim, n, N, J, M, prec in (first, second):
        log(f"fine_propagate_noalloc dim={dim} n={n} N={N} J={J} M={M} prec={prec}")
        w = (W.small_1d if dim == 1 else W.small_2d)(n=n, N=N, J=J)
        a, starts, want, got = _case(ctx, w, M, prec, 7 + n)
        assert torch.equal(got, want)
        g = host(got)
        for m in range(M):
            P = prop.Propagators(dim, n, a[m], w.T, N, J, w.forcing)
            for s in range(N):
                assert rel(g[m, s], P.F(starts[m, s])) < 1e-11


def test_noalloc_honours_the_active_mask(ctx):
    w = W.small_2d(n=33, N=4, J=3)
    log("fine_propagate_noalloc with an active mask")
    _, _, want, got = _case(ctx, w, 3, 1, 5, active=[1, 0, 1])
    assert torch.equal(got, want)
    assert (host(got)[1] == -3.0).all()


def test_noalloc_rejects_a_workspace_beyond_the_array(ctx):
    import paper_2510_26180_amd as K
    # 2 x 8 B increments x 128^2 unknowns x 8 samples x 64 slices = 134 MB > 64 MiB
    w = W.small_2d(n=128, N=64, J=1)
    M = 8
    log("fine_propagate_noalloc beyond its scratch array")
    a = dev(oracle_faces(w, W.draw_xi(M, w.d, 3)))
    start = torch.zeros((M, w.N, w.Nx), dtype=torch.float64, device="cuda")
    end = torch.full_like(start, -3.0)
    with pytest.raises(K.KlecgcError) as e:
        ctx.fine_propagate_noalloc(spec_of(w, precision=1), a, start, end)
    assert e.value.code == -1 and "scratch" in str(e.value)
    assert bool((end == -3.0).all())
    # the context's own workspace is untouched by the failed call: a regular call still works
    small = W.small_2d(n=16, N=2, J=2)
    a2, s2, want, got = _case(ctx, small, 1, 1, 9)
    assert torch.equal(got, want)
