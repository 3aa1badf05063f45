"""rnmf_hals_step_noalloc (the sweeps without a workspace, for callers that
cannot allocate) against rnmf_hals_step on the same inputs, through the C
ABI: two calls in a row, the second on a smaller problem, each bit-identical
to the workspace entry point (same kernel, same launch shape, deterministic
exchange), with a clean device status; and a problem too large for the fixed
scratch is refused before any launch."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
rn = pytest.importorskip("paper_1711_02037_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not rn.available():
        raise RuntimeError("librnmf.so is not built")


def _problem(m, n, k, l, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    Q, _ = torch.linalg.qr(torch.randn(m, l, generator=g, dtype=torch.float64))
    X = torch.rand(m, k, generator=g, dtype=torch.float64) @ torch.rand(k, n, generator=g, dtype=torch.float64)
    B = Q.T @ X
    W0 = torch.rand(m, k, generator=g, dtype=torch.float64)
    H0 = torch.rand(k, n, generator=g, dtype=torch.float64)
    Wt0 = Q.T @ W0
    return [t.float().contiguous().to(DEV) for t in (Q, B, W0, Wt0, H0)]


@pytest.mark.parametrize("shapes", [[(20000, 3000, 32, 48, 1), (5000, 700, 12, 30, 2)]])
def test_noalloc_matches_workspace_entry_point_twice(shapes):
    for (m, n, k, l, seed) in shapes:
        Q, B, W0, Wt0, H0 = _problem(m, n, k, l, seed)
        W1, Wt1, H1 = W0.clone(), Wt0.clone(), H0.clone()
        r1 = rn.hals_step(Q, B, W1, Wt1, H1, nsweeps=3)
        W2, Wt2, H2 = W0.clone(), Wt0.clone(), H0.clone()
        r2 = rn.hals_step_noalloc(Q, B, W2, Wt2, H2, nsweeps=3)
        torch.cuda.synchronize()
        assert r2[0] == r1[0] == 3
        assert r2[3] == 0
        for a, b in ((W2, W1), (Wt2, Wt1), (H2, H1)):
            assert torch.equal(a, b)
        # a different start through the same scratch: still identical
        W3, Wt3, H3 = (W0 * 0.5).contiguous(), (Wt0 * 0.5).contiguous(), H0.clone()
        W4, Wt4, H4 = W3.clone(), Wt3.clone(), H3.clone()
        rn.hals_step(Q, B, W3, Wt3, H3, nsweeps=2, tol=1e-12)
        r4 = rn.hals_step_noalloc(Q, B, W4, Wt4, H4, nsweeps=2, tol=1e-12)
        assert r4[3] == 0
        assert torch.equal(W3, W4) and torch.equal(H3, H4) and torch.equal(Wt3, Wt4)


def test_noalloc_refuses_a_problem_beyond_its_scratch():
    L = rn.lib()
    m, n, k, l = 100000, 5000, 64, 128
    o = rn.make_opts(k, l - k, 0)
    p = ctypes.c_void_p(256)  # never dereferenced: the size check comes first
    st = L.rnmf_hals_step_noalloc(p, p, m, n, l, k, p, p, p, 1, ctypes.byref(o), None, None, None)
    assert st == rn.ERR_WORKSPACE
    assert b"bytes of scratch" in L.rnmf_last_error()
