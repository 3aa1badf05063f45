"""GPU parity: every C-ABI entry point against the FP64 oracle on identical,
seeded inputs.  The oracle receives the device inputs promoted to float64.

Tolerances (per step, from identical inputs):
  FP32: relative Frobenius error <= 1e-5 for B, W, W~, H after one sweep;
        orthogonality ||Q^T Q - I||_F <= 1e-5 and range capture within 1e-5
        (relative) of the oracle's; final relative error within 1e-4 absolute.
  FP64: 1e-12 for Q-related quantities and compression, 1e-10 for sweeps and
        the final error.
Q itself is compared column by column only in FP64: in FP32 the trailing
columns of Q move by about cond(Y) * 2^-24, which is legitimate.
"""

import math

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


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    return t.detach().to("cpu").to(torch.float64).numpy()


def relf(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def problem(m, n, rank, k, p, seed, noise=0.01, dtype=np.float32):
    X, Om, W0, H0 = s.random_problem(m, n, rank, k, p, seed, noise_abs=noise)
    return X.astype(dtype), Om.astype(dtype), W0.astype(dtype), H0.astype(dtype)


# ---------------------------------------------------------------------------
# Range finder and compression
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,k,p,q", [(500, 400, 10, 20, 2), (333, 517, 7, 9, 1), (1000, 64, 5, 11, 0)])
def test_sketch_fp64_matches_oracle_q(m, n, k, p, q):
    X, Om, _, _ = problem(m, n, 10, k, p, 11, dtype=np.float64)
    Q = rn.sketch(dev(X), k, p, q, omega=dev(Om), precision="fp64")
    Qo = o.range_finder(X, Om, q)
    Qg = host(Q)
    assert np.linalg.norm(Qg.T @ Qg - np.eye(Qg.shape[1])) <= 1e-12
    # canonical thin QR (positive diag R): Q columns agree, loosened by cond(Y)
    assert np.max(np.abs(Qg - Qo)) <= 1e-9


@pytest.mark.parametrize("m,n,k,p,q", [(4000, 700, 16, 20, 2), (3001, 1025, 50, 20, 2), (257, 129, 3, 5, 1),
                                       (5000, 2410, 16, 20, 2)])
def test_sketch_fp32_orthonormal_and_captures_range(m, n, k, p, q):
    X, Om, _, _ = problem(m, n, 40, k, p, 12)
    Q = rn.sketch(dev(X), k, p, q, omega=dev(Om), precision="fp32")
    Qg = host(Q)
    l = Qg.shape[1]
    assert np.linalg.norm(Qg.T @ Qg - np.eye(l)) <= 1e-5
    X64 = X.astype(np.float64)
    Qo = o.range_finder(X64, Om.astype(np.float64), q)
    cap_g = np.linalg.norm(X64 - Qg @ (Qg.T @ X64)) / np.linalg.norm(X64)
    cap_o = np.linalg.norm(X64 - Qo @ (Qo.T @ X64)) / np.linalg.norm(X64)
    assert abs(cap_g - cap_o) <= 1e-5 * max(cap_o, 1e-3) + 1e-6
    # same subspace as the oracle's (leading directions agree)
    assert np.linalg.norm(Qo.T @ Qg, 2) <= 1 + 1e-5


def test_sketch_with_strided_input_and_generated_omega():
    m, n, k, p = 600, 300, 8, 8
    X, _, _, _ = problem(m, n, 10, k, p, 13)
    big = np.zeros((m, n + 7), np.float32)
    big[:, :n] = X
    Xd = dev(big)[:, :n]
    assert Xd.stride(0) == n + 7
    Q1 = rn.sketch(Xd, k, p, 1, seed=5)
    Q2 = rn.sketch(dev(X), k, p, 1, seed=5)
    # a different row stride selects a different load width (and summation
    # grouping): the bases agree in the subspace they capture, not entry-wise
    X64 = X.astype(np.float64)
    cap = [np.linalg.norm(X64 - Qa @ (Qa.T @ X64)) / np.linalg.norm(X64) for Qa in (host(Q1), host(Q2))]
    assert abs(cap[0] - cap[1]) <= 1e-5 * cap[1]
    assert torch.equal(Q2, rn.sketch(dev(X), k, p, 1, seed=5))
    Qg = host(Q1)
    assert np.linalg.norm(Qg.T @ Qg - np.eye(k + p)) <= 1e-5


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp64", 1e-12)])
@pytest.mark.parametrize("m,n,l", [(500, 400, 30), (3001, 1025, 70), (129, 2411, 17)])
def test_compress_matches_oracle(prec, tol, m, n, l):
    dt = np.float64 if prec == "fp64" else np.float32
    X, _, _, _ = problem(m, n, 10, 5, 5, 14, dtype=dt)
    Qn, _ = np.linalg.qr(s.stream(14, 1).standard_normal((m, l)))
    Qd = dev(Qn.astype(dt))
    B = rn.compress(dev(X), Qd, precision=prec)
    Bo = o.compress(X.astype(np.float64), host(Qd))
    assert relf(host(B), Bo) <= tol


# ---------------------------------------------------------------------------
# Sweeps from identical inputs
# ---------------------------------------------------------------------------

def sweep_inputs(m, n, k, l, seed, dt):
    X, Om, W0, H0 = problem(m, n, max(k, 4), k, l - k, seed, dtype=np.float64)
    Q = o.range_finder(X, Om, 1)
    B = Q.T @ X
    Wt = Q.T @ W0
    return [a.astype(dt) for a in (Q, B, W0, Wt, H0)]


@pytest.mark.parametrize("gram", ["full", "lowdim", "mixed"])
@pytest.mark.parametrize("order", ["h_first", "w_first"])
@pytest.mark.parametrize("m,n,k,l", [(1000, 300, 10, 30), (5003, 1711, 50, 70), (40, 33, 3, 8),
                                     (20000, 3000, 40, 84), (3001, 1025, 50, 96)])  # Q slab of 12 columns a lane
def test_hals_step_one_sweep_fp32(gram, order, m, n, k, l):
    Q, B, W, Wt, H = sweep_inputs(m, n, k, l, 21, np.float32)
    d = [dev(a) for a in (Q, B, W, Wt, H)]
    done, _, _ = rn.hals_step(*d, nsweeps=1, gram=gram, order=order)
    assert done == 1
    Wo, Wto, Ho = o.rhals_sweep(*(a.astype(np.float64) for a in (Q, B, W, Wt, H)),
                                gram_mode=rn.GRAM[gram], order=rn.ORDER[order])
    assert relf(host(d[2]), Wo) <= 1e-5
    assert relf(host(d[3]), Wto) <= 1e-5
    assert relf(host(d[4]), Ho) <= 1e-5
    assert host(d[2]).min() >= 0 and host(d[4]).min() >= 0


@pytest.mark.parametrize("m,n,k,l,tol", [(3000, 900, 20, 100, 0.0),      # l > 72: Q slab in LDS
                                          (120000, 200, 8, 16, 0.0),     # > 448 rows per workgroup
                                          (3000, 900, 20, 100, 1e-12)])  # with the stopping test
def test_hals_step_lds_slab_path(m, n, k, l, tol):
    Q, B, W, Wt, H = sweep_inputs(m, n, k, l, 27, np.float32)
    d = [dev(a) for a in (Q, B, W, Wt, H)]
    done, _, _ = rn.hals_step(*d, nsweeps=2, tol=tol)
    assert done == 2
    a = tuple(x.astype(np.float64) for x in (Q, B, W, Wt, H))
    for _ in range(2):
        a = a[:2] + o.rhals_sweep(*a)
    assert relf(host(d[2]), a[2]) <= 2e-5
    assert relf(host(d[3]), a[3]) <= 2e-5
    assert relf(host(d[4]), a[4]) <= 2e-5


@pytest.mark.parametrize("gram,tol", [("full", 0.0), ("lowdim", 0.0), ("mixed", 0.0), ("full", 1e-12)])
@pytest.mark.parametrize("m,n,k,l", [(100000, 600, 64, 84), (99991, 257, 60, 80)])
def test_hals_step_w_global_path(gram, tol, m, n, k, l):
    # Q slab in registers with the W rows in global memory: the rows of W
    # (about 400 per workgroup at this k) do not fit in LDS beside the rest
    plan = rn.sweep_plan(m, n, l, k, tol=tol)
    assert plan["q_slab"] == "registers" and plan["w_global"], plan
    Q, B, W, Wt, H = sweep_inputs(m, n, k, l, 23, np.float32)
    d = [dev(a) for a in (Q, B, W, Wt, H)]
    done, _, _ = rn.hals_step(*d, nsweeps=2, gram=gram, tol=tol)
    assert done == 2
    a = tuple(x.astype(np.float64) for x in (Q, B, W, Wt, H))
    for _ in range(2):
        a = a[:2] + o.rhals_sweep(*a, gram_mode=rn.GRAM[gram])
    assert relf(host(d[2]), a[2]) <= 2e-5
    assert relf(host(d[3]), a[3]) <= 2e-5
    assert relf(host(d[4]), a[4]) <= 2e-5
    assert host(d[2]).min() >= 0 and host(d[4]).min() >= 0


def test_sweep_plan_paths():
    # the headline shape keeps W in LDS; the LDS-slab path beyond 448 rows
    p = rn.sweep_plan(100000, 5000, 70, 50)
    assert p["q_slab"] == "registers" and not p["w_global"] and p["owners"] > 0
    p = rn.sweep_plan(120000, 200, 16, 8)
    assert p["q_slab"] == "lds"
    p = rn.sweep_plan(100000, 5000, 84, 64)
    assert p["q_slab"] == "registers" and p["w_global"]


@pytest.mark.parametrize("gram", ["full", "lowdim", "mixed"])
def test_hals_step_fp64_ten_sweeps(gram):
    Q, B, W, Wt, H = sweep_inputs(500, 400, 10, 30, 22, np.float64)
    d = [dev(a) for a in (Q, B, W, Wt, H)]
    rn.hals_step(*d, nsweeps=10, gram=gram)
    a = (Q, B, W, Wt, H)
    for _ in range(10):
        a = (Q, B) + o.rhals_sweep(*a, gram_mode=rn.GRAM[gram])
    assert relf(host(d[2]), a[2]) <= 1e-10
    assert relf(host(d[3]), a[3]) <= 1e-10
    assert relf(host(d[4]), a[4]) <= 1e-10


def test_hals_step_ten_sweeps_fp32_tracks_oracle():
    Q, B, W, Wt, H = sweep_inputs(3000, 800, 16, 36, 23, np.float32)
    d = [dev(a) for a in (Q, B, W, Wt, H)]
    rn.hals_step(*d, nsweeps=10)
    a = tuple(x.astype(np.float64) for x in (Q, B, W, Wt, H))
    for _ in range(10):
        a = a[:2] + o.rhals_sweep(*a)
    assert relf(host(d[2]), a[2]) <= 1e-4
    assert relf(host(d[4]), a[4]) <= 1e-4


def test_hals_step_skips_zero_scale_blocks():
    Q, B, W, Wt, H = sweep_inputs(800, 300, 6, 16, 24, np.float64)
    H[2, :] = 0.0   # V_22 = 0
    W[:, 4] = 0.0   # S_44 = 0
    Wt = Q.T @ W
    d = [dev(a) for a in (Q, B, W, Wt, H)]
    rn.hals_step(*d, nsweeps=1)
    Wo, Wto, Ho = o.rhals_sweep(Q, B, W, Wt, H)
    assert relf(host(d[2]), Wo) <= 1e-10
    assert relf(host(d[4]), Ho) <= 1e-10
    assert np.all(np.isfinite(host(d[2])))


def test_hals_step_tolerance_stops_like_oracle():
    Q, B, W, Wt, H = sweep_inputs(400, 300, 5, 12, 25, np.float64)
    d = [dev(a) for a in (Q, B, W, Wt, H)]
    done, pg0, pg = rn.hals_step(*d, nsweeps=500, tol=1e-3)
    a = (Q, B, W, Wt, H)
    pg0o = o.projected_gradient_sq_compressed(*a)
    assert abs(pg0 - pg0o) <= 1e-10 * pg0o
    it = 0
    while it < 500:
        a = (Q, B) + o.rhals_sweep(*a)
        it += 1
        if o.projected_gradient_sq_compressed(*a) < 1e-3 * pg0o:
            break
    assert done == it
    assert relf(host(d[2]), a[2]) <= 1e-9


def test_hals_step_is_deterministic():
    Q, B, W, Wt, H = sweep_inputs(5003, 1711, 50, 70, 26, np.float32)
    outs = []
    for _ in range(2):
        d = [dev(a) for a in (Q, B, W, Wt, H)]
        rn.hals_step(*d, nsweeps=3)
        outs.append([t.clone() for t in d[2:]])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


# ---------------------------------------------------------------------------
# End to end
# ---------------------------------------------------------------------------

def test_factorize_fp64_small_matches_oracle():
    X, Om, W0, H0, w = s.make("small_500x400")
    W, H, info = rn.factorize(dev(X), w["k"], w["p"], w["q"], max_iter=w["sweeps"], precision="fp64",
                              omega=dev(Om), W0=dev(W0), H0=dev(H0))
    Wo, Ho, io = o.rhals(X, w["k"], Om, W0, H0, q=w["q"], max_iter=w["sweeps"])
    assert info["iters"] == 100
    assert abs(info["rel_err"] - io["rel_err"]) <= 1e-10
    assert relf(host(W), Wo) <= 1e-8 and relf(host(H), Ho) <= 1e-8
    # compressed error ||B - W~ H|| / ||B|| on the oracle's own B, W~, H
    comp_o = np.linalg.norm(io["B"] - io["Wt"] @ Ho) / np.linalg.norm(io["B"])
    assert abs(info["comp_err"] - comp_o) <= 1e-9


@pytest.mark.parametrize("m,n,k,p,sweeps", [(2000, 700, 12, 20, 60), (777, 1301, 20, 10, 40)])
def test_factorize_fp32_final_error_matches_oracle(m, n, k, p, sweeps):
    X, Om, W0, H0 = problem(m, n, 30, k, p, 31)
    W, H, info = rn.factorize(dev(X), k, p, 2, max_iter=sweeps, omega=dev(Om), W0=dev(W0), H0=dev(H0))
    Wo, Ho, io = o.rhals(X.astype(np.float64), k, Om.astype(np.float64), W0.astype(np.float64),
                         H0.astype(np.float64), q=2, max_iter=sweeps)
    assert abs(info["rel_err"] - io["rel_err"]) <= 1e-4
    assert abs(info["rel_err"] - o.rel_error(X.astype(np.float64), host(W), host(H))) <= 1e-6
    comp_o = np.linalg.norm(io["B"] - io["Wt"] @ Ho) / np.linalg.norm(io["B"])
    assert abs(info["comp_err"] - comp_o) <= 1e-4
    assert host(W).min() >= 0 and host(H).min() >= 0


def test_factorize_bf16_form_error_against_oracle():
    m, n, k, p = 4000, 1200, 16, 20
    X, Om, W0, H0 = problem(m, n, 30, k, p, 32)
    W, H, info = rn.factorize(dev(X), k, p, 2, max_iter=80, precision="bf16", omega=dev(Om), W0=dev(W0),
                              H0=dev(H0))
    _, _, io = o.rhals(X.astype(np.float64), k, Om.astype(np.float64), W0.astype(np.float64),
                       H0.astype(np.float64), q=3, max_iter=80)
    assert info["q"] == 3
    # BF16 rounds X by up to 2^-9; per-step parity is unpinned for this form,
    # the final error must stay within 1% of the oracle's
    assert info["rel_err"] <= 1.01 * io["rel_err"]
    assert abs(info["rel_err"] - o.rel_error(X.astype(np.float64), host(W), host(H))) <= 1e-6


def test_bf16_sketch_is_orthonormal():
    X, Om, _, _ = problem(5000, 2410, 40, 16, 20, 33)
    Q = rn.sketch(dev(X), 16, 20, 3, omega=dev(Om), precision="bf16", exact_q=True)
    Qg = host(Q)
    assert np.linalg.norm(Qg.T @ Qg - np.eye(36)) <= 1e-6


def test_factorize_generated_init_is_reproducible_and_nonnegative():
    X, _, _, _ = problem(1500, 900, 20, 10, 10, 34)
    a = rn.factorize(dev(X), 10, 10, 2, max_iter=20, seed=99)
    b = rn.factorize(dev(X), 10, 10, 2, max_iter=20, seed=99)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert host(a[0]).min() >= 0 and host(a[1]).min() >= 0
    assert a[2]["rel_err"] < 0.2


def test_factorize_clipped_gaussian_init():
    """init="gauss" (the Remark on initialization after Algorithm 1): with
    max_iter = 0 the factorization returns its start, which must be standard
    normal entries with the negative ones set to zero: about half exactly
    zero, the rest a half-normal sample (Kolmogorov-Smirnov at 1e-3), the
    same for the same seed and different from the uniform start; from that
    start the sweeps follow the oracle's."""
    from scipy import stats
    X, Om, _, _ = problem(1500, 900, 20, 10, 10, 37, dtype=np.float64)
    W, H, _ = rn.factorize(dev(X), 10, 10, 2, max_iter=0, seed=5, precision="fp64", omega=dev(Om), init="gauss")
    W2, H2, _ = rn.factorize(dev(X), 10, 10, 2, max_iter=0, seed=5, precision="fp64", omega=dev(Om), init="gauss")
    Wu, _, _ = rn.factorize(dev(X), 10, 10, 2, max_iter=0, seed=5, precision="fp64", omega=dev(Om))
    assert torch.equal(W, W2) and torch.equal(H, H2) and not torch.equal(W, Wu)
    v = np.concatenate([host(W).ravel(), host(H).ravel()])
    N = v.size
    zero = np.count_nonzero(v == 0.0)
    assert v.min() >= 0.0
    assert abs(zero - N / 2) <= 5 * np.sqrt(N / 4)
    assert stats.kstest(v[v > 0], stats.halfnorm.cdf).pvalue > 1e-3
    W0, H0 = host(W), host(H)
    Wg, Hg, info = rn.factorize(dev(X), 10, 10, 2, max_iter=30, seed=5, precision="fp64", omega=dev(Om),
                                init="gauss")
    Wo, Ho, io = o.rhals(X, 10, Om, W0, H0, q=2, max_iter=30)
    assert abs(info["rel_err"] - io["rel_err"]) <= 1e-10
    assert relf(host(Wg), Wo) <= 1e-8 and relf(host(Hg), Ho) <= 1e-8


def test_factorize_stops_on_tolerance():
    X, Om, W0, H0 = problem(1200, 500, 6, 6, 10, 35, dtype=np.float64)
    W, H, info = rn.factorize(dev(X), 6, 10, 2, max_iter=2000, tol=1e-4, precision="fp64", omega=dev(Om),
                              W0=dev(W0), H0=dev(H0))
    _, _, io = o.rhals(X, 6, Om, W0, H0, q=2, max_iter=2000, tol=1e-4)
    assert info["iters"] == io["iters"] < 2000
    assert abs(info["pg_ratio"] - io["pg_ratio"]) <= 1e-8


# ---------------------------------------------------------------------------
# Errors found on the device
# ---------------------------------------------------------------------------

def test_negative_and_nonfinite_input_are_reported():
    X, _, _, _ = problem(300, 200, 5, 4, 4, 36)
    Xn = X.copy(); Xn[7, 9] = -1.0
    with pytest.raises(rn.RnmfError) as e:
        rn.factorize(dev(Xn), 4, 4, 1, max_iter=2)
    assert e.value.status == rn.ERR_NEGATIVE_INPUT
    Xf = X.copy(); Xf[3, 3] = np.nan
    with pytest.raises(rn.RnmfError) as e:
        rn.factorize(dev(Xf), 4, 4, 1, max_iter=2, precision="bf16")
    assert e.value.status == rn.ERR_NONFINITE
    # the BF16 form scans X while it makes the bfloat16 copy
    with pytest.raises(rn.RnmfError) as e:
        rn.factorize(dev(Xn), 4, 4, 1, max_iter=2, precision="bf16")
    assert e.value.status == rn.ERR_NEGATIVE_INPUT


def test_exactly_low_rank_input_gives_a_valid_basis():
    # Y = X Omega has rank 3 < l = 8: the Gram matrix is singular, and Cholesky
    # QR must still return an orthonormal basis that captures range(X)
    # (through the shifted pass when the unshifted factorisation breaks down).
    m, n, r = 400, 300, 3
    g = s.stream(37, 0)
    X = (g.random((m, r)) @ g.random((r, n))).astype(np.float64)
    Q = host(rn.sketch(dev(X), 3, 5, 1, precision="fp64", seed=3))
    assert np.linalg.norm(X - Q @ (Q.T @ X)) / np.linalg.norm(X) <= 1e-10
    W, H, info = rn.factorize(dev(X), 3, 5, 1, max_iter=300, precision="fp64", seed=3)
    assert host(W).min() >= 0 and host(H).min() >= 0
    assert info["rel_err"] < 1e-3


def test_exactly_low_rank_fp32_gives_a_valid_basis():
    # rank 3 < l = 8 in FP32: rounding in Y = X Omega keeps the Gram numerically
    # positive definite, and Cholesky QR2 still returns an orthonormal basis
    # that captures range(X) to FP32 accuracy.
    m, n, r = 3000, 500, 3
    g = s.stream(41, 0)
    X = (g.random((m, r)) @ g.random((r, n))).astype(np.float32)
    Q = host(rn.sketch(dev(X), 3, 5, 1, precision="fp32", seed=5))
    l = Q.shape[1]
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) <= 1e-5
    Xd = X.astype(np.float64)
    assert np.linalg.norm(Xd - Q @ (Q.T @ Xd)) / np.linalg.norm(Xd) <= 1e-5


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_shifted_cholesky_qr3_matches_oracle_basis(prec, tol):
    # shifted pass first, then two plain passes (the third runs in place):
    # the basis is the same thin QR, so it spans the oracle's subspace
    m, n, k, p, q = 4000, 900, 12, 8, 1
    dt = np.float64 if prec == "fp64" else np.float32
    X, Om, _, _ = problem(m, n, 20, k, p, 45, dtype=dt)
    Q = host(rn.sketch(dev(X), k, p, q, omega=dev(Om), precision=prec, shift="always"))
    Qo = o.range_finder(X.astype(np.float64), Om.astype(np.float64), q)
    l = Q.shape[1]
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) <= tol
    assert np.linalg.norm(Q @ Q.T @ Qo - Qo) / np.linalg.norm(Qo) <= 100 * tol
    _, _, info = rn.factorize(dev(X), k, p, q, max_iter=3, precision=prec, omega=dev(Om), shift="always")
    assert info["shifted_qr"]


def test_well_conditioned_sketch_needs_no_shift():
    X, Om, W0, H0 = problem(2000, 700, 10, 10, 10, 43)
    _, _, info = rn.factorize(dev(X), 10, 10, 1, max_iter=2, precision="fp32", omega=dev(Om), W0=dev(W0),
                              H0=dev(H0))
    assert not info["shifted_qr"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("m,n,ld,k,p", [(500, 400, 400, 10, 20), (3001, 2410, 2432, 16, 20),
                                        (5003, 1711, 1728, 50, 20), (20007, 333, 384, 8, 8)])
def test_sketch_pass_spans_x_omega(prec, m, n, ld, k, p):
    # with q = 0, Q = qr(X Omega): every column of X Omega (computed here in
    # FP64 from the same rounded inputs) must lie in span(Q).  An error in the
    # streamed product (a lost tail, a wrong split or tile) shows up directly.
    # Shapes: ragged m, ragged n inside a padded row (ld > n), one to several
    # reduction splits.
    g = s.stream(47, m, n)
    Xf = np.zeros((m, ld), dtype=np.float32)
    Xf[:, :n] = g.random((m, n), dtype=np.float32)
    Xf[:, n:] = np.nan                       # padding must never be read as data
    l = s.sketch_cols(k, p, m, n)
    Om = g.standard_normal((n, l)).astype(np.float32)
    Xd = dev(Xf)
    if prec == "bf16":
        Xd = Xd.to(torch.bfloat16)[:, :n]     # round to nearest even, padded rows
        Xh = host(Xd)
    else:
        Xd = Xd[:, :n]
        Xh = Xf[:, :n].astype(np.float64)
    # exact_q: the BF16 form would otherwise add one subspace iteration
    Q = host(rn.sketch(Xd, k, p, 0, omega=dev(Om), precision=prec, exact_q=True))
    # the BF16 sketch pass takes Omega rounded to bfloat16 (nearest even)
    Omh = host(dev(Om).to(torch.bfloat16)) if prec == "bf16" else Om.astype(np.float64)
    Y = Xh @ Omh
    err = np.linalg.norm(Y - Q @ (Q.T @ Y)) / np.linalg.norm(Y)
    assert err <= 2e-6, err
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("m,n,ld,l", [(500, 400, 400, 30), (3001, 1711, 1728, 70), (20007, 333, 336, 28),
                                      (4099, 5000, 5000, 70)])
def test_compress_streamed_shapes(prec, m, n, ld, l):
    # B = Q^T X against the product in FP64 of the same rounded inputs:
    # ragged m and n, n inside padded rows whose padding is NaN (never data),
    # several column blocks and row splits
    g = s.stream(53, m, n)
    Xf = np.full((m, ld), np.nan, dtype=np.float32)
    Xf[:, :n] = g.random((m, n), dtype=np.float32)
    Qn, _ = np.linalg.qr(g.standard_normal((m, l)))
    Qn = Qn.astype(np.float32)
    Xd = dev(Xf)
    Xd = (Xd.to(torch.bfloat16) if prec == "bf16" else Xd)[:, :n]
    B = host(rn.compress(Xd, dev(Qn), precision=prec))
    Bo = Qn.astype(np.float64).T @ host(Xd)
    assert np.isfinite(B).all()
    assert relf(B, Bo) <= 1e-5


# n % 4 == 0 takes the 16-byte loads of X in the matrix-core kernel (at least
# 128 row tiles), the other widths its element loads, the small shapes the
# tiled kernel
@pytest.mark.parametrize("m,n,k", [(1000, 300, 10), (3001, 2411, 50), (20007, 333, 7), (100000, 130, 64),
                                   (50, 40, 3), (3001, 2412, 50), (4099, 1000, 33), (100000, 132, 64),
                                   (2048, 4, 1)])
def test_rel_error_matches_fp64(m, n, k):
    g = s.stream(71, m, n)
    X = g.random((m, n), dtype=np.float32)
    W = g.random((m, k), dtype=np.float32)
    H = (g.random((k, n), dtype=np.float32) / k).astype(np.float32)
    e = rn.rel_error(dev(X), dev(W), dev(H))
    Xd = X.astype(np.float64)
    eo = np.linalg.norm(Xd - W.astype(np.float64) @ H.astype(np.float64)) / np.linalg.norm(Xd)
    assert abs(e - eo) <= 1e-6 * eo
