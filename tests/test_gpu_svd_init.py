"""GPU parity of the SVD-based initialization (rnmf_svd_init; the Remark on
initialization after Algorithm 1, reading R20) against the FP64 oracle's
svd_init on identical Q and B.

Bars.  FP32: W and H within 1e-5 relative Frobenius.  Rounding Q and B to FP32
moves the oracle's own result by 2e-8 to 9e-8 on these shapes, and the device
works in FP64 from there.  FP64: 1e-8.  The device takes the singular
vectors of B from Jacobi on B B^T, whose eigenvector error is about
eps ||B||^2 / (sigma_j^2 - sigma_{j+1}^2); the closest leading singular values
here are 4e-6 sigma_1 apart.  In every case the choice between positive and
negative parts has a relative margin of at least 6e-4, far above either
rounding, so both sides take the same decisions.
"""

import numpy as np
import pytest

import oracle as o
import synth as s

torch = pytest.importorskip("torch")
rn = pytest.importorskip("paper_1711_02037_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not rn.available():
        raise RuntimeError("librnmf.so is not built")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().to("cpu").to(torch.float64).numpy()


def relf(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def qb_inputs(m, n, k, l, seed):
    X, Om, _, _ = s.random_problem(m, n, max(k, 4) + 20, k, l - k, seed, noise_abs=0.01)
    Q = o.range_finder(X, Om, 1)
    return X, Q, Q.T @ X


SHAPES = [(500, 400, 10, 30, 501),     # several 64-row blocks, ragged tails
          (3001, 1025, 50, 70, 502),   # the performance-study sketch width
          (777, 300, 7, 96, 503),      # the largest supported l
          (2000, 700, 12, 31, 504),    # odd l: one index sits out each round
          (100, 1500, 5, 20, 505)]     # wide: more columns than rows


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-5)])
@pytest.mark.parametrize("m,n,k,l,seed", SHAPES)
def test_svd_init_matches_oracle(prec, tol, m, n, k, l, seed):
    _, Q, B = qb_inputs(m, n, k, l, seed)
    dt = np.float64 if prec == "fp64" else np.float32
    Qd, Bd = dev(Q.astype(dt)), dev(B.astype(dt))
    W, H = rn.svd_init(Qd, Bd, k)
    Wo, Ho = o.svd_init(host(Qd), host(Bd), k)
    Wh, Hh = host(W), host(H)
    assert Wh.min() >= 0.0 and Hh.min() >= 0.0
    assert relf(Wh, Wo) <= tol and relf(Hh, Ho) <= tol
    # the zero pattern is the oracle's wherever the oracle's entry is clearly nonzero
    big = np.abs(Wo) > 1e-6 * np.abs(Wo).max()
    assert np.all(Wh[big] > 0.0)


def test_svd_init_is_deterministic():
    _, Q, B = qb_inputs(3001, 1025, 50, 70, 506)
    Qd, Bd = dev(Q.astype(np.float32)), dev(B.astype(np.float32))
    a = rn.svd_init(Qd, Bd, 50)
    b = rn.svd_init(Qd, Bd, 50)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_factorize_with_svd_init_fp64_matches_oracle():
    X, Om, _, _ = s.random_problem(600, 450, 25, 10, 20, 507, noise_abs=0.01)
    W, H, info = rn.factorize(dev(X), 10, 20, 2, max_iter=50, precision="fp64", omega=dev(Om), init="svd")
    Qo, Bo = o.qb(X, Om, 2)
    W0, H0 = o.svd_init(Qo, Bo, 10)
    Wo, Ho, io = o.rhals(X, 10, Om, W0, H0, q=2, max_iter=50)
    assert abs(info["rel_err"] - io["rel_err"]) <= 1e-9
    assert relf(host(W), Wo) <= 1e-7 and relf(host(H), Ho) <= 1e-7


def test_factorize_with_svd_init_fp32_final_error_matches_oracle():
    m, n, k, p, sweeps = 2000, 700, 12, 20, 60
    X, Om, _, _ = s.random_problem(m, n, 30, k, p, 508, noise_abs=0.01)
    X32, Om32 = X.astype(np.float32), Om.astype(np.float32)
    W, H, info = rn.factorize(dev(X32), k, p, 2, max_iter=sweeps, omega=dev(Om32), init="svd")
    Xd, Omd = X32.astype(np.float64), Om32.astype(np.float64)
    Qo, Bo = o.qb(Xd, Omd, 2)
    W0, H0 = o.svd_init(Qo, Bo, k)
    _, _, io = o.rhals(Xd, k, Omd, W0, H0, q=2, max_iter=sweeps)
    assert abs(info["rel_err"] - io["rel_err"]) <= 1e-4
    assert host(W).min() >= 0 and host(H).min() >= 0
