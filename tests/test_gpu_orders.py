"""GPU parity of compressed-HALS sweeps with an explicit order of block
updates (rnmf_hals_ordered; Sec. 3.2's interleaved and blocked orders and the
shuffled order, reading R24) against the oracle's rhals_sweep_ordered on the
same inputs.

Bars as for rnmf_hals_step: FP32 one sweep <= 1e-5 relative Frobenius per
factor, from the same FP32 inputs; FP64 three sweeps <= 1e-10.  The blocked
lists are also checked against the persistent sweep kernel, which runs the
same updates with other sums (FP64: 1e-10).
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


def dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(DEV)


def host(t):
    return t.detach().to("cpu").to(torch.float64).numpy()


def relf(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(m, n, k, l, seed, dt):
    X = s.low_rank_rows(m, n, k + 2, seed, noise_abs=0.02)
    Q = o.range_finder(X, s.omega(n, l, seed), 1)
    W0, H0 = s.init_factors(m, n, k, seed)
    r = lambda a: a.astype(dt).astype(np.float64)
    Q, W0, H0 = r(Q), r(W0), r(H0)
    B = r(Q.T @ X)
    Wt0 = r(Q.T @ W0)
    return Q, B, W0, Wt0, H0


def orders_for(kind, k, nsw, seed):
    if kind == "interleaved":
        return [rn.order_interleaved(k) for _ in range(nsw)]
    if kind == "shuffled":
        g = s.stream(seed, 56)
        return [rn.order_interleaved(k, g.permutation(k)) for _ in range(nsw)]
    if kind == "blocked_h":
        return [rn.order_blocked(k) for _ in range(nsw)]
    if kind == "blocked_w":
        return [rn.order_blocked(k, True) for _ in range(nsw)]
    raise ValueError(kind)


def run(Q, B, W0, Wt0, H0, orders, dt):
    Qd, Bd = dev(Q, dt), dev(B, dt)
    W, Wt, H = dev(W0, dt), dev(Wt0, dt), dev(H0, dt)
    rn.hals_ordered(Qd, Bd, W, Wt, H, orders)
    torch.cuda.synchronize()
    return host(W), host(Wt), host(H)


def oracle_run(Q, B, W0, Wt0, H0, orders):
    W, Wt, H = W0, Wt0, H0
    for od in orders:
        W, Wt, H = o.rhals_sweep_ordered(Q, B, W, Wt, H, od)
    return W, Wt, H


SHAPES = [(700, 520, 6, 14, 701),     # ragged 256-row and 128-column blocks
          (3001, 1025, 50, 70, 702),  # the performance-study sketch width
          (300, 200, 1, 1, 703),      # k = l = 1
          (1000, 300, 40, 128, 704)]  # the largest l


@pytest.mark.parametrize("kind", ["interleaved", "shuffled", "blocked_h", "blocked_w"])
@pytest.mark.parametrize("m,n,k,l,seed", SHAPES)
def test_ordered_sweeps_fp64(kind, m, n, k, l, seed):
    print(f"case fp64 {kind} m={m} n={n} k={k} l={l}", flush=True)
    Q, B, W0, Wt0, H0 = problem(m, n, k, l, seed, np.float64)
    orders = orders_for(kind, k, 3, seed)
    got = run(Q, B, W0, Wt0, H0, orders, np.float64)
    ref = oracle_run(Q, B, W0, Wt0, H0, orders)
    errs = [relf(a, b) for a, b in zip(got, ref)]
    assert max(errs) <= 1e-10, errs


@pytest.mark.parametrize("kind", ["interleaved", "shuffled", "blocked_w"])
@pytest.mark.parametrize("m,n,k,l,seed", SHAPES[:2])
def test_ordered_sweep_fp32(kind, m, n, k, l, seed):
    print(f"case fp32 {kind} m={m} n={n} k={k} l={l}", flush=True)
    Q, B, W0, Wt0, H0 = problem(m, n, k, l, seed, np.float32)
    orders = orders_for(kind, k, 1, seed)
    got = run(Q, B, W0, Wt0, H0, orders, np.float32)
    ref = oracle_run(Q, B, W0, Wt0, H0, orders)
    errs = [relf(a, b) for a, b in zip(got, ref)]
    print("fp32 errors W Wt H", errs, flush=True)
    assert max(errs) <= 1e-5, errs


@pytest.mark.parametrize("w_first", [False, True])
def test_blocked_lists_match_the_sweep_kernel(w_first):
    m, n, k, l, seed = 2000, 900, 12, 30, 711
    Q, B, W0, Wt0, H0 = problem(m, n, k, l, seed, np.float64)
    got = run(Q, B, W0, Wt0, H0, [rn.order_blocked(k, w_first)] * 3, np.float64)
    Qd, Bd = dev(Q, np.float64), dev(B, np.float64)
    W, Wt, H = dev(W0, np.float64), dev(Wt0, np.float64), dev(H0, np.float64)
    rn.hals_step(Qd, Bd, W, Wt, H, nsweeps=3, order="w_first" if w_first else "h_first")
    torch.cuda.synchronize()
    errs = [relf(a, host(b)) for a, b in zip(got, (W, Wt, H))]
    assert max(errs) <= 1e-10, errs


def test_zero_scale_blocks_are_skipped():
    # component 1 starts at zero: V_11 = 0 skips column 1 of W, and then
    # S_11 = 0 skips row 1 of H, in every sweep
    m, n, k, l, seed = 500, 300, 5, 12, 712
    Q, B, W0, Wt0, H0 = problem(m, n, k, l, seed, np.float64)
    H0 = H0.copy(); H0[1, :] = 0.0
    W0 = W0.copy(); W0[:, 1] = 0.0
    Wt0 = Q.T @ W0
    orders = [rn.order_blocked(k, True), rn.order_interleaved(k), rn.order_blocked(k)]
    got = run(Q, B, W0, Wt0, H0, orders, np.float64)
    ref = oracle_run(Q, B, W0, Wt0, H0, orders)
    errs = [relf(a, b) for a, b in zip(got, ref)]
    assert max(errs) <= 1e-10, errs
    assert not got[0][:, 1].any() and not got[2][1, :].any()
