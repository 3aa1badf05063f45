"""Pins for the FP64 oracle: each check ties an oracle function to a fact that
does not come from the oracle's own formula (a closed form, a textbook or
library routine, a brute-force minimiser, an independent implementation,
finite differences, an inequality the mathematics fixes)."""

import math
import os
import warnings

import numpy as np
import pytest

import oracle as o
import synth as s

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def _rand(seed, *shape):
    return s.stream(seed, 99).random(shape)


def _exact_low_rank(m, n, r, seed):
    g = s.stream(seed, 0)
    return g.random((m, r)) @ g.random((r, n))


# ---------------------------------------------------------------------------
# QR and the range finder (Sec. 2.3; Algorithm 1)
# ---------------------------------------------------------------------------

def test_qr_positive_is_the_unique_cholesky_qr():
    # For full-rank Y the thin QR with positive diag(R) is unique; it must equal
    # the factor built from the Cholesky factor of the Gram matrix.
    Y = _rand(1, 40, 7) + 0.1
    Q, R = o.qr_positive(Y)
    L = np.linalg.cholesky(Y.T @ Y)
    Q2 = np.linalg.solve(L, Y.T).T
    assert np.allclose(Q, Q2, atol=1e-12)
    assert np.allclose(R, L.T, atol=1e-12)
    assert np.all(np.diag(R) >= 0)
    assert np.allclose(np.triu(R), R)
    assert np.allclose(Q @ R, Y, atol=1e-13)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_exact_capture_of_low_rank_range(q):
    # X of exact rank r <= l: Q Q^T X = X (closed form of the QB scheme).
    m, n, r, l = 300, 200, 8, 12
    X = _exact_low_rank(m, n, r, 7)
    Om = s.omega(n, l, 7)
    Q = o.range_finder(X, Om, q)
    assert Q.shape == (m, l)
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) <= 1e-13
    err = np.linalg.norm(X - Q @ (Q.T @ X)) / np.linalg.norm(X)
    assert err <= 1e-13


@pytest.mark.parametrize("q", [1, 2])
def test_subspace_iteration_equals_direct_power_scheme(q):
    # In exact arithmetic the re-orthonormalised subspace iteration returns the
    # same canonical Q as the QR of ((X X^T)^q X) Omega; on a well-conditioned
    # small problem the two agree entry by entry.
    X = _rand(3, 40, 30)
    Om = s.omega(30, 5, 3)
    Y = X @ Om
    for _ in range(q):
        Y = X @ (X.T @ Y)
    Qd, _ = o.qr_positive(Y)
    assert np.allclose(o.range_finder(X, Om, q), Qd, atol=1e-9)


def test_qb_error_bounds():
    # Eckart-Young gives ||X - QB||_2 >= sigma_{l+1}; the expected-error bound
    # of Sec. 2.3 bounds the mean over independent test matrices.
    m, n, k, p = 200, 150, 10, 5
    U, _ = np.linalg.qr(s.stream(5, 0).standard_normal((m, n)))
    V, _ = np.linalg.qr(s.stream(5, 1).standard_normal((n, n)))
    sig = 0.7 ** np.arange(n)
    X = (U * sig) @ V.T
    l = k + p
    for q in (0, 1, 2):
        errs = []
        for seed in range(20):
            Om = s.omega(n, l, 1000 + seed)
            Q, B = o.qb(X, Om, q)
            e = np.linalg.norm(X - Q @ B, 2)
            assert e >= sig[l] * (1 - 1e-9)
            errs.append(e)
        bound = (1 + math.sqrt(k / (p - 1)) + math.e * math.sqrt(k + p) / p
                 * math.sqrt(n - k)) ** (1.0 / (2 * q + 1)) * sig[k]
        assert np.mean(errs) <= bound


def test_streaming_qb_spans_the_same_subspace():
    # Algorithm 2 (column-streamed) and Algorithm 1 build the same subspace.
    m, n, l = 120, 90, 8
    X = _rand(11, m, n) + _exact_low_rank(m, n, 4, 11)
    Om = s.omega(n, l, 11)
    for q in (0, 1, 2):
        Q1, B1 = o.qb(X, Om, q)
        Q2, B2 = o.qb_streaming(X, Om, q, block=7)
        assert np.linalg.norm(Q1 @ Q1.T - Q2 @ Q2.T, 2) <= 1e-8
        assert np.allclose(Q1 @ B1, Q2 @ B2, atol=1e-8)


def test_compress_projects_onto_basis():
    X = _exact_low_rank(50, 40, 3, 4)
    Q = o.range_finder(X, s.omega(40, 6, 4), 1)
    B = o.compress(X, Q)
    assert B.shape == (6, 40)
    assert np.allclose(Q @ B, X, atol=1e-12)


# ---------------------------------------------------------------------------
# HALS sweeps (Sec. 3.1) against independent minimisers
# ---------------------------------------------------------------------------

def _nnls_1col(w, R):
    # argmin_{h >= 0} ||R - w h^T||_F, column by column, by scipy's NNLS.
    from scipy.optimize import nnls
    A = w.reshape(-1, 1)
    return np.array([nnls(A, R[:, c])[0][0] for c in range(R.shape[1])])


def test_hals_sweep_equals_blockwise_nnls_on_explicit_residual():
    # Each HALS block update is the exact nonnegative least-squares minimiser of
    # the explicit residual R^(j) (Sec. 3.1, Eqs. hals and residual).
    m, n, k = 9, 7, 3
    X = _rand(21, m, n)
    W = _rand(22, m, k)
    H = _rand(23, k, n)
    Wn, Hn = o.hals_sweep(X, W, H, o.ORDER_H_FIRST)
    Wb, Hb = W.copy(), H.copy()
    for j in range(k):
        Rj = X - Wb @ Hb + np.outer(Wb[:, j], Hb[j, :])
        Hb[j, :] = _nnls_1col(Wb[:, j], Rj)
    for j in range(k):
        Rj = X - Wb @ Hb + np.outer(Wb[:, j], Hb[j, :])
        Wb[:, j] = _nnls_1col(Hb[j, :], Rj.T)
    assert np.allclose(Hn, Hb, atol=1e-10)
    assert np.allclose(Wn, Wb, atol=1e-10)


def test_hals_matches_scikit_learn_coordinate_descent():
    # scikit-learn's coordinate-descent NMF runs cyclic HALS with the W block
    # first; with the same start and no regularisation the iterates agree.
    nmf = pytest.importorskip("sklearn.decomposition._nmf")
    m, n, k = 30, 25, 4
    X = _rand(31, m, n)
    W0 = _rand(32, m, k)
    H0 = _rand(33, k, n)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        Ws, Hs, it = nmf._fit_coordinate_descent(X, W0.copy(), H0.copy(), tol=0.0,
                                                  max_iter=25, shuffle=False)
    Wo, Ho, info = o.hals(X, W0, H0, max_iter=25, order=o.ORDER_W_FIRST)
    assert it == 25 and info["iters"] == 25
    assert np.allclose(Wo, Ws, rtol=1e-10, atol=1e-12)
    assert np.allclose(Ho, Hs, rtol=1e-10, atol=1e-12)


def test_hals_objective_is_monotone():
    # Every block update is an exact minimiser, so f never increases.
    X = s.low_rank_rows(40, 30, 5, 41, noise_abs=0.05)
    W, H = s.init_factors(40, 30, 4, 41)
    f = np.linalg.norm(X - W @ H) ** 2
    for order in (o.ORDER_H_FIRST, o.ORDER_W_FIRST):
        Wc, Hc, fc = W.copy(), H.copy(), f
        for _ in range(60):
            Wc, Hc = o.hals_sweep(X, Wc, Hc, order)
            fn = np.linalg.norm(X - Wc @ Hc) ** 2
            assert fn <= fc * (1 + 1e-12)
            fc = fn


@pytest.mark.parametrize("seed", [2, 3])
def test_exact_low_rank_reaches_near_machine_precision(seed):
    # Sec. 4.4: on exactly low-rank nonnegative data both HALS and rHALS fit the
    # data to nearly machine precision (seeds 2 and 3 are the ones recorded).
    m, n, r = 60, 50, 3
    g = s.stream(1000 + seed, 0)
    X = g.random((m, r)) @ g.random((r, n))
    W0, H0 = s.init_factors(m, n, r, 2000 + seed)
    _, _, ih = o.hals(X, W0, H0, max_iter=3000)
    Om = s.omega(n, r + 5, 3000 + seed)
    Wr, Hr, ir = o.rhals(X, r, Om, W0, H0, q=1, max_iter=3000)
    assert ih["rel_err"] <= 1e-10
    assert ir["rel_err"] <= 1e-10
    assert Wr.min() >= 0 and Hr.min() >= 0


def test_rank_one_is_the_perron_singular_pair():
    # With k = 1 HALS is an alternating power method: W H converges to
    # sigma_1 u_1 v_1^T (LAPACK SVD; Perron vectors are nonnegative).
    X = s.low_rank_rows(40, 30, 3, 51, noise_abs=0.02)
    W0, H0 = s.init_factors(40, 30, 1, 51)
    W, H, info = o.hals(X, W0, H0, max_iter=400)
    U, sv, Vt = np.linalg.svd(X)
    best = sv[0] * np.outer(U[:, 0], Vt[0])
    assert np.linalg.norm(W @ H - best) / np.linalg.norm(best) <= 1e-10
    assert abs(info["rel_err"] - math.sqrt(np.sum(sv[1:] ** 2)) / np.linalg.norm(X)) <= 1e-10
    assert info["pg_ratio"] <= 1e-12
    # rHALS with k = 1 is the same power method on X^ = Q B.
    Om = s.omega(30, 6, 51)
    Wr, Hr, ir = o.rhals(X, 1, Om, W0, H0, q=2, max_iter=400)
    Xh = ir["Q"] @ ir["B"]
    U, sv, Vt = np.linalg.svd(Xh)
    best = sv[0] * np.outer(U[:, 0], Vt[0])
    assert np.linalg.norm(Wr @ Hr - best) / np.linalg.norm(best) <= 1e-10


def test_kkt_residual_vanishes_at_convergence():
    m, n, r = 60, 50, 3
    g = s.stream(1003, 0)
    X = g.random((m, r)) @ g.random((r, n))
    W0, H0 = s.init_factors(m, n, r, 2003)
    W, H, info = o.hals(X, W0, H0, max_iter=3000)
    assert info["pg_ratio"] <= 1e-12
    assert W.min() >= 0 and H.min() >= 0


# ---------------------------------------------------------------------------
# Randomized HALS sweep (Sec. 3.2; Algorithm 1)
# ---------------------------------------------------------------------------

def _rhals_setup(seed, m=30, n=24, k=3, l=7):
    X = s.low_rank_rows(m, n, 4, seed, noise_abs=0.05)
    Q = o.range_finder(X, s.omega(n, l, seed), 1)
    B = Q.T @ X
    W0, H0 = s.init_factors(m, n, k, seed)
    return X, Q, B, W0, Q.T @ W0, H0


def test_rhals_sweep_equals_explicit_compressed_minimisers():
    # H rows: with S = W^T W the H rule is the NNLS minimiser on the explicit
    # residual of X^ = Q B with the true W.  W~ columns: the unconstrained
    # least-squares minimiser of the compressed residual (Eqs. rhals and
    # residualLD), then lift, clip and map back (Sec. 3.2).
    X, Q, B, W, Wt, H = _rhals_setup(61)
    Wn, Wtn, Hn = o.rhals_sweep(Q, B, W, Wt, H)
    Xh = Q @ B
    k = H.shape[0]
    Wb, Wtb, Hb = W.copy(), Wt.copy(), H.copy()
    for j in range(k):
        Rj = Xh - Wb @ Hb + np.outer(Wb[:, j], Hb[j, :])
        Hb[j, :] = _nnls_1col(Wb[:, j], Rj)
    for j in range(k):
        Rt = B - Wtb @ Hb + np.outer(Wtb[:, j], Hb[j, :])
        w, *_ = np.linalg.lstsq(Hb[j, :].reshape(-1, 1), Rt.T, rcond=None)
        Wb[:, j] = np.maximum(Q @ w.ravel(), 0.0)
        Wtb[:, j] = Q.T @ Wb[:, j]
    assert np.allclose(Hn, Hb, atol=1e-10)
    assert np.allclose(Wn, Wb, atol=1e-10)
    assert np.allclose(Wtn, Wtb, atol=1e-10)


def test_rhals_sweep_lowdim_gram_is_compressed_minimiser():
    # GRAM_LOWDIM: the H rule printed in Sec. 3.2 is the NNLS minimiser of the
    # compressed residual B - sum_{i != j} W~_i H_i.
    X, Q, B, W, Wt, H = _rhals_setup(62)
    Wn, Wtn, Hn = o.rhals_sweep(Q, B, W, Wt, H, gram_mode=o.GRAM_LOWDIM)
    Hb = H.copy()
    for j in range(H.shape[0]):
        Rt = B - Wt @ Hb + np.outer(Wt[:, j], Hb[j, :])
        Hb[j, :] = _nnls_1col(Wt[:, j], Rt)
    assert np.allclose(Hn, Hb, atol=1e-10)


def test_rhals_sweep_mixed_gram_is_proximal_compressed_minimiser():
    # GRAM_MIXED (the note after the rHALS H rule in Sec. 3.2): numerator from
    # the compressed Gram W~^T W~, scale (W^T W)_jj.  That update is the exact
    # minimiser over h >= 0 of the compressed residual cost plus a proximal
    # term, 1/2 ||Rt - w~_j h^T||^2 + 1/2 rho ||h - h_old||^2 with
    # rho = ||w_j||^2 - ||w~_j||^2 >= 0 (the part of W(:,j) outside range(Q)).
    # Solved here per column by scipy's NNLS on the stacked system
    # [w~_j; sqrt(rho)] h = [Rt(:, c); sqrt(rho) h_old(c)].  Swapping the
    # numerator and the scale (or using one Gram for both) fails it, because
    # W has a large component outside range(Q) in this setup.
    from scipy.optimize import nnls
    X, Q, B, W, Wt, H = _rhals_setup(65)
    Wn, Wtn, Hn = o.rhals_sweep(Q, B, W, Wt, H, gram_mode=o.GRAM_MIXED)
    k = H.shape[0]
    Hb = H.copy()
    for j in range(k):
        rho = W[:, j] @ W[:, j] - Wt[:, j] @ Wt[:, j]
        assert rho > 0.1 * (W[:, j] @ W[:, j])  # the pin separates the Grams
        Rt = B - Wt @ Hb + np.outer(Wt[:, j], Hb[j, :])
        A = np.concatenate([Wt[:, j], [math.sqrt(rho)]]).reshape(-1, 1)
        Hb[j, :] = [nnls(A, np.concatenate([Rt[:, c], [math.sqrt(rho) * Hb[j, c]]]))[0][0]
                    for c in range(Hb.shape[1])]
    assert np.allclose(Hn, Hb, atol=1e-10)
    # the W phase does not depend on the Gram mode
    Wf, Wtf, _ = o.rhals_sweep(Q, B, W, Wt, Hb, order=o.ORDER_W_FIRST)
    Wm, Wtm, _ = o.rhals_sweep(Q, B, W, Wt, Hb, gram_mode=o.GRAM_MIXED, order=o.ORDER_W_FIRST)
    assert np.array_equal(Wf, Wm) and np.array_equal(Wtf, Wtm)


def test_rhals_full_space_equivalent_form():
    # In m-space, the W~ step plus lift equals W_j <- [P_Q (W_j + (X^ H^T_j -
    # W V_j) / V_jj)]_+ with P_Q = Q Q^T, which holds because W~ = Q^T W.
    m, n, k, l = 60, 40, 4, 9
    X = s.low_rank_rows(m, n, 5, 63, noise_abs=0.05)
    Q = o.range_finder(X, s.omega(n, l, 63), 2)
    B = Q.T @ X
    W, H = s.init_factors(m, n, k, 63)
    Wt = Q.T @ W
    Xh = Q @ B
    P = Q @ Q.T
    Wf, Hf = W.copy(), H.copy()
    for _ in range(5):
        W, Wt, H = o.rhals_sweep(Q, B, W, Wt, H)
        S = Wf.T @ Wf
        G = Xh.T @ Wf
        for j in range(k):
            Hf[j] = np.maximum(Hf[j] + (G[:, j] - Hf.T @ S[:, j]) / S[j, j], 0)
        V = Hf @ Hf.T
        XH = Xh @ Hf.T
        for j in range(k):
            Wf[:, j] = np.maximum(P @ (Wf[:, j] + (XH[:, j] - Wf @ V[:, j]) / V[j, j]), 0)
    assert np.allclose(W, Wf, atol=1e-12)
    assert np.allclose(H, Hf, atol=1e-12)


@pytest.mark.parametrize("gram", [o.GRAM_FULL, o.GRAM_LOWDIM, o.GRAM_MIXED])
def test_rhals_is_basis_invariant(gram):
    # Replacing Q by Q U (U orthogonal) rotates B and W~ by U^T and leaves W, H
    # unchanged.
    X, Q, B, W, Wt, H = _rhals_setup(64)
    U, _ = np.linalg.qr(s.stream(64, 7).standard_normal((Q.shape[1],) * 2))
    Q2, B2, Wt2 = Q @ U, U.T @ B, U.T @ Wt
    a = (W, Wt, H)
    b = (W, Wt2, H)
    for _ in range(4):
        a = o.rhals_sweep(Q, B, *a, gram_mode=gram)
        b = o.rhals_sweep(Q2, B2, *b, gram_mode=gram)
    assert np.allclose(a[0], b[0], atol=1e-12)
    assert np.allclose(a[2], b[2], atol=1e-12)
    assert np.allclose(U @ b[1], a[1], atol=1e-12)


def test_rhals_with_identity_basis_is_hals():
    # With Q = I (l = m) the compressed sweep is the deterministic sweep; with a
    # random orthogonal Q of full width it is HALS in a rotated frame.
    m, n, k = 12, 30, 3
    X = _rand(71, m, n)
    W, H = s.init_factors(m, n, k, 71)
    for order in (o.ORDER_H_FIRST, o.ORDER_W_FIRST):
        Wh, Hh = o.hals_sweep(X, W, H, order)
        Wr, _, Hr = o.rhals_sweep(np.eye(m), X, W, W.copy(), H, order=order)
        assert np.array_equal(Wh, Wr) and np.array_equal(Hh, Hr)
        U, _ = np.linalg.qr(s.stream(71, 1).standard_normal((m, m)))
        Wu, _, Hu = o.rhals_sweep(U, U.T @ X, W, U.T @ W, H, order=order)
        assert np.allclose(Wu, Wh, atol=1e-12) and np.allclose(Hu, Hh, atol=1e-12)


def test_zero_scale_blocks_are_skipped():
    X, Q, B, W, Wt, H = _rhals_setup(72)
    H[1, :] = 0.0           # V_11 = 0: W step 1 must be skipped
    W[:, 2] = 0.0           # S_22 = 0: H row 2 must be skipped
    Wt = Q.T @ W
    Wn, Wtn, Hn = o.rhals_sweep(Q, B, W, Wt, H)
    assert np.all(np.isfinite(Wn)) and np.all(np.isfinite(Hn))
    assert np.array_equal(Hn[2], H[2])


# ---------------------------------------------------------------------------
# Stopping measure and error (Sec. 3.3)
# ---------------------------------------------------------------------------

def test_projected_gradient_matches_finite_differences():
    m, n, k = 6, 5, 2
    X = _rand(81, m, n)
    W = _rand(82, m, k) + 0.1
    H = _rand(83, k, n) + 0.1

    def f(W, H):
        return np.sum((X - W @ H) ** 2)

    h = 1e-6
    gW = np.zeros_like(W)
    gH = np.zeros_like(H)
    for idx in np.ndindex(W.shape):
        E = np.zeros_like(W); E[idx] = h
        gW[idx] = (f(W + E, H) - f(W - E, H)) / (2 * h)
    for idx in np.ndindex(H.shape):
        E = np.zeros_like(H); E[idx] = h
        gH[idx] = (f(W, H + E) - f(W, H - E)) / (2 * h)
    # interior point: projection is the identity; factor 2 is dropped
    pg = o.projected_gradient_sq(X, W, H)
    assert abs(pg - (np.sum(gW ** 2) + np.sum(gH ** 2)) / 4) <= 1e-7 * pg
    # on the boundary only descent directions count
    W0 = W.copy(); W0[0, 0] = 0.0
    gW0 = gW.copy()
    for idx in np.ndindex(W.shape):
        E = np.zeros_like(W); E[idx] = h
        gW0[idx] = (f(W0 + E, H) - f(W0 - E, H)) / (2 * h)
    gW0[0, 0] = min(gW0[0, 0], 0.0)
    gH0 = np.zeros_like(H)
    for idx in np.ndindex(H.shape):
        E = np.zeros_like(H); E[idx] = h
        gH0[idx] = (f(W0, H + E) - f(W0, H - E)) / (2 * h)
    pg0 = o.projected_gradient_sq(X, W0, H)
    assert abs(pg0 - (np.sum(gW0 ** 2) + np.sum(gH0 ** 2)) / 4) <= 1e-7 * pg0


def test_compressed_projected_gradient_is_gradient_on_surrogate():
    X, Q, B, W, Wt, H = _rhals_setup(84)
    W[0, 0] = 0.0
    Wt = Q.T @ W
    a = o.projected_gradient_sq_compressed(Q, B, W, Wt, H)
    b = o.projected_gradient_sq(Q @ B, W, H)
    assert abs(a - b) <= 1e-12 * b


def test_rel_error_special_cases():
    X = _rand(91, 8, 6)
    W = _rand(92, 8, 2)
    H = _rand(93, 2, 6)
    assert o.rel_error(W @ H, W, H) <= 1e-15
    assert o.rel_error(X, np.zeros((8, 2)), H) == pytest.approx(1.0, abs=1e-15)
    assert o.rel_error(2 * X, W, H) == pytest.approx(
        math.sqrt(np.sum((2 * X - W @ H) ** 2) / np.sum(4 * X * X)), rel=1e-13)


def test_clip_maps_nonpositive_to_positive_zero():
    c = o.clip(np.array([-1.0, -0.0, 0.0, 2.0]))
    assert list(c) == [0.0, 0.0, 0.0, 2.0]
    assert not np.signbit(c).any()


# ---------------------------------------------------------------------------
# Drivers (Algorithm 1 end to end) and the paper's quality claim
# ---------------------------------------------------------------------------

def test_rhals_driver_runs_sweeps_and_stops_on_tolerance():
    X, Om, W0, H0 = s.random_problem(80, 60, 5, 4, 6, 101)
    W, H, info = o.rhals(X, 4, Om, W0, H0, q=2, max_iter=7)
    Q, B = o.qb(X, Om, 2)
    a = (W0, Q.T @ W0, H0)
    for _ in range(7):
        a = o.rhals_sweep(Q, B, *a)
    assert info["iters"] == 7
    assert np.allclose(W, a[0], atol=1e-13) and np.allclose(H, a[2], atol=1e-13)
    W2, H2, i2 = o.rhals(X, 4, Om, W0, H0, q=2, max_iter=10000, tol=1e-6)
    assert i2["iters"] < 10000 and i2["pg_ratio"] < 1e-6
    assert W2.min() >= 0 and H2.min() >= 0


@pytest.mark.parametrize("seed", [101, 103])
def test_rhals_error_tracks_deterministic_hals(seed):
    # Sec. 4, Tables 1-3: run to a tight projected-gradient tolerance, rHALS
    # reaches the error of deterministic HALS to about three digits.
    X, Om, W0, H0 = s.random_problem(200, 150, 5, 5, 10, seed, noise_abs=0.01)
    _, _, ih = o.hals(X, W0, H0, max_iter=5000, tol=1e-10)
    _, _, ir = o.rhals(X, 5, Om, W0, H0, q=2, max_iter=5000, tol=1e-10)
    assert ih["iters"] < 5000 and ir["iters"] < 5000
    assert abs(ir["rel_err"] - ih["rel_err"]) <= 1e-2 * ih["rel_err"]


def test_argument_checks():
    X, Om, W0, H0 = s.random_problem(20, 15, 3, 3, 2, 5)
    with pytest.raises(ValueError):
        o.rhals(X, 15, Om, W0, H0)
    with pytest.raises(ValueError):
        o.rhals_sweep(np.eye(20), X, W0, W0, H0, gram_mode=7)
    assert o.sketch_width(10, 20, 500, 400) == 30
    assert o.sketch_width(10, 20, 500, 25) == 25
