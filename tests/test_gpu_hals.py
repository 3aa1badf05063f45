"""GPU parity of deterministic HALS (rnmf_hals; Sec. 3.1) against the FP64
oracle's hals_sweep on identical inputs (the oracle receives the device inputs
promoted to float64).

Tolerances: one FP32 sweep, W and H each within 1e-5 relative (Frobenius);
FP64, ten sweeps within 1e-10.  At the full 100,000 x 5,000 size the FP32
bar is 1e-4: R = X^T W and T = X H^T are FP32 matrix-core sums over 5,000
and 100,000 terms (relative error up to about sqrt(n) u = 4e-6 per entry),
and the update's numerator T - W V cancels most of T, which multiplies that
error several times over.  (Randomized HALS meets 1e-5 at this size because
its T and V are formed with FP64 accumulation over only l rows.)  The objective of deterministic HALS is
non-increasing sweep by sweep (each block update is an exact minimiser), which
is checked on the device result at full size.
"""

import os

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


def problem(m, n, k, seed, dt):
    X, _, W0, H0 = s.random_problem(m, n, max(k, 4), k, 0, seed, noise_abs=0.01)
    return X.astype(dt), W0.astype(dt), H0.astype(dt)


@pytest.mark.parametrize("order", ["h_first", "w_first"])
@pytest.mark.parametrize("m,n,k", [(1000, 300, 10), (5003, 1711, 50), (40, 33, 3), (3001, 2410, 64)])
def test_hals_one_sweep_fp32(order, m, n, k):
    X, W0, H0 = problem(m, n, k, 61, np.float32)
    W, H = dev(W0), dev(H0)
    rn.hals(dev(X), W, H, nsweeps=1, order=order)
    Wo, Ho = o.hals_sweep(X.astype(np.float64), W0.astype(np.float64), H0.astype(np.float64),
                          order=o.ORDER_W_FIRST if order == "w_first" else o.ORDER_H_FIRST)
    assert relf(host(W), Wo) <= 1e-5
    assert relf(host(H), Ho) <= 1e-5


def test_hals_fp64_ten_sweeps():
    X, W0, H0 = problem(700, 500, 12, 62, np.float64)
    W, H = dev(W0), dev(H0)
    rn.hals(dev(X), W, H, nsweeps=10)
    Wo, Ho = W0.copy(), H0.copy()
    for _ in range(10):
        Wo, Ho = o.hals_sweep(X, Wo, Ho)
    assert relf(host(W), Wo) <= 1e-10
    assert relf(host(H), Ho) <= 1e-10


def test_hals_skips_zero_scale_blocks():
    # an all-zero row of H and an all-zero column of W have zero scale; the
    # oracle skips their updates, so must the device
    X, W0, H0 = problem(600, 400, 6, 63, np.float32)
    H0[2, :] = 0.0
    W0[:, 4] = 0.0
    W, H = dev(W0), dev(H0)
    rn.hals(dev(X), W, H, nsweeps=1)
    Wo, Ho = o.hals_sweep(X.astype(np.float64), W0.astype(np.float64), H0.astype(np.float64))
    assert relf(host(W), Wo) <= 1e-5
    assert relf(host(H), Ho) <= 1e-5


def test_hals_full_size_sweep_and_monotone_objective():
    # the tall performance-study workload (100,000 x 5,000, k = 50): one sweep
    # against the oracle, then the objective over further sweeps
    X, Om, W0, H0, w = s.make("tall_100000x5000", threads=min(16, os.cpu_count() or 1))
    Xd = dev(X)
    W, H = dev(W0), dev(H0)
    rn.hals(Xd, W, H, nsweeps=1)
    Wo, Ho = o.hals_sweep(X.astype(np.float64), W0.astype(np.float64), H0.astype(np.float64))
    assert relf(host(W), Wo) <= 1e-4
    assert relf(host(H), Ho) <= 1e-4
    errs = [rn.rel_error(Xd, W, H)]
    for _ in range(5):
        rn.hals(Xd, W, H, nsweeps=1)
        errs.append(rn.rel_error(Xd, W, H))
    assert all(b <= a * (1 + 1e-6) for a, b in zip(errs, errs[1:])), errs
