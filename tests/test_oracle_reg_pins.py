"""Pins for the regularized HALS rules of the oracle (Sec. 3.4 and its
appendix; readings R18 and R19).  Each check ties the rules to a fact outside
their own formula: scikit-learn's coordinate-descent NMF (which applies the
same ridge and LASSO terms), brute-force minimisers of the per-block cost,
finite differences of the cost, monotone descent, first-order optimality at
convergence, and the reduction of the compressed sweep to the deterministic one
when the basis is square and orthogonal."""

import warnings

import numpy as np
import pytest

import oracle as o
import synth as s

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")

REGS = {
    "ridge": o.Reg(alpha_w=0.7, alpha_h=0.3),
    "lasso": o.Reg(beta_w=0.05, beta_h=0.2),
    "elastic": o.Reg(alpha_w=0.4, alpha_h=0.9, beta_w=0.1, beta_h=0.03),
}


def _rand(seed, *shape):
    return s.stream(seed, 99).random(shape)


@pytest.mark.parametrize("name", sorted(REGS))
def test_regularized_hals_matches_scikit_learn_coordinate_descent(name):
    # scikit-learn adds the ridge weight to the Gram diagonal and subtracts the
    # LASSO weight from the cross product before its cyclic coordinate updates
    # (W block first); those are the printed rules of Sec. 3.4.
    nmf = pytest.importorskip("sklearn.decomposition._nmf")
    r = REGS[name]
    m, n, k = 30, 25, 4
    X = _rand(131, m, n)
    W0 = _rand(132, m, k)
    H0 = _rand(133, k, n)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        Ws, Hs, it = nmf._fit_coordinate_descent(
            X, W0.copy(), H0.copy(), tol=0.0, max_iter=20, l1_reg_W=r.beta_w, l1_reg_H=r.beta_h,
            l2_reg_W=r.alpha_w, l2_reg_H=r.alpha_h, shuffle=False)
    Wo, Ho, info = o.hals(X, W0, H0, max_iter=20, order=o.ORDER_W_FIRST, reg=r)
    assert it == 20 and info["iters"] == 20
    assert np.allclose(Wo, Ws, rtol=1e-10, atol=1e-12)
    assert np.allclose(Ho, Hs, rtol=1e-10, atol=1e-12)


def _block_cost_min(w, Rj, alpha, beta):
    """argmin over h >= 0 of 1/2 ||Rj - w h^T||^2 + alpha/2 ||h||^2 + beta sum(h),
    entry by entry with scipy's bounded scalar minimiser (no closed form)."""
    from scipy.optimize import minimize_scalar
    ww = float(w @ w)
    out = np.empty(Rj.shape[1])
    for c in range(Rj.shape[1]):
        col = Rj[:, c]

        def f(h):
            e = col - w * h
            return 0.5 * float(e @ e) + 0.5 * alpha * h * h + beta * h

        ub = 10.0 * (abs(float(w @ col)) + 1.0) / (ww + alpha + 1e-300)
        res = minimize_scalar(f, bounds=(0.0, ub), method="bounded", options={"xatol": 1e-13})
        out[c] = res.x if f(res.x) < f(0.0) else 0.0
    return out


@pytest.mark.parametrize("name", sorted(REGS))
def test_regularized_sweep_equals_brute_force_block_minimisers(name):
    r = REGS[name]
    m, n, k = 9, 7, 3
    X = _rand(141, m, n)
    W = _rand(142, m, k)
    H = _rand(143, k, n)
    Wn, Hn = o.hals_sweep(X, W, H, o.ORDER_H_FIRST, reg=r)
    Wb, Hb = W.copy(), H.copy()
    for j in range(k):
        Rj = X - Wb @ Hb + np.outer(Wb[:, j], Hb[j, :])
        Hb[j, :] = _block_cost_min(Wb[:, j], Rj, r.alpha_h, r.beta_h)
    for j in range(k):
        Rj = X - Wb @ Hb + np.outer(Wb[:, j], Hb[j, :])
        Wb[:, j] = _block_cost_min(Hb[j, :], Rj.T, r.alpha_w, r.beta_w)
    assert np.allclose(Hn, Hb, atol=1e-8)
    assert np.allclose(Wn, Wb, atol=1e-8)


@pytest.mark.parametrize("name", sorted(REGS))
def test_regularized_objective_is_monotone(name):
    r = REGS[name]
    X = s.low_rank_rows(40, 30, 5, 151, noise_abs=0.05)
    W, H = s.init_factors(40, 30, 4, 151)
    for order in (o.ORDER_H_FIRST, o.ORDER_W_FIRST):
        Wc, Hc = W.copy(), H.copy()
        fc = o.objective(X, Wc, Hc, r)
        for _ in range(60):
            Wc, Hc = o.hals_sweep(X, Wc, Hc, order, reg=r)
            fn = o.objective(X, Wc, Hc, r)
            assert fn <= fc * (1 + 1e-12)
            fc = fn


def test_regularized_gradient_matches_finite_differences_of_the_cost():
    # At an interior point the projected gradient is the gradient of the cost
    # that the rules minimise, 1/2 ||X - W H||^2 + alpha/2 ||F||^2 + beta sum(F).
    r = REGS["elastic"]
    m, n, k = 6, 5, 2
    X = _rand(161, m, n)
    W = _rand(162, m, k) + 0.1
    H = _rand(163, k, n) + 0.1
    h = 1e-6
    gW = np.zeros_like(W)
    gH = np.zeros_like(H)
    for idx in np.ndindex(W.shape):
        E = np.zeros_like(W); E[idx] = h
        gW[idx] = (o.objective(X, W + E, H, r) - o.objective(X, W - E, H, r)) / (2 * h)
    for idx in np.ndindex(H.shape):
        E = np.zeros_like(H); E[idx] = h
        gH[idx] = (o.objective(X, W, H + E, r) - o.objective(X, W, H - E, r)) / (2 * h)
    pg = o.projected_gradient_sq(X, W, H, r)
    assert abs(pg - (np.sum(gW ** 2) + np.sum(gH ** 2))) <= 1e-7 * pg
    # the cost itself: 1-norm of nonnegative factors and the ridge term
    e = X - W @ H
    f = 0.5 * np.sum(e ** 2) + 0.5 * r.alpha_w * np.linalg.norm(W) ** 2 + r.beta_w * np.abs(W).sum() \
        + 0.5 * r.alpha_h * np.linalg.norm(H) ** 2 + r.beta_h * np.abs(H).sum()
    assert abs(o.objective(X, W, H, r) - f) <= 1e-12 * f


@pytest.mark.parametrize("name", sorted(REGS))
def test_regularized_kkt_residual_vanishes_at_convergence(name):
    r = REGS[name]
    X = s.low_rank_rows(50, 40, 3, 171, noise_abs=0.02)
    W0, H0 = s.init_factors(50, 40, 3, 171)
    W, H, info = o.hals(X, W0, H0, max_iter=4000, reg=r)
    assert info["pg_ratio"] <= 1e-12
    assert W.min() >= 0 and H.min() >= 0


def test_zero_weights_reproduce_the_plain_rules_bit_for_bit():
    X = s.low_rank_rows(30, 24, 4, 181, noise_abs=0.05)
    Q = o.range_finder(X, s.omega(24, 7, 181), 1)
    B = Q.T @ X
    W, H = s.init_factors(30, 24, 3, 181)
    for order in (o.ORDER_H_FIRST, o.ORDER_W_FIRST):
        a = o.rhals_sweep(Q, B, W, Q.T @ W, H, order=order)
        b = o.rhals_sweep(Q, B, W, Q.T @ W, H, order=order, reg=o.Reg())
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
        a = o.hals_sweep(X, W, H, order)
        b = o.hals_sweep(X, W, H, order, reg=o.Reg(0.0, 0.0, 0.0, 0.0))
        assert all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("name", sorted(REGS))
def test_regularized_rhals_with_square_orthogonal_basis_is_regularized_hals(name):
    # Reading R19: with Q square and orthogonal the compressed sweep, whose
    # LASSO shift is applied after the lift, is the deterministic sweep.
    r = REGS[name]
    m, n, k = 12, 30, 3
    X = _rand(191, m, n)
    W, H = s.init_factors(m, n, k, 191)
    for order in (o.ORDER_H_FIRST, o.ORDER_W_FIRST):
        Wh, Hh = o.hals_sweep(X, W, H, order, reg=r)
        Wr, _, Hr = o.rhals_sweep(np.eye(m), X, W, W.copy(), H, order=order, reg=r)
        assert np.allclose(Wr, Wh, atol=1e-12) and np.allclose(Hr, Hh, atol=1e-12)
        U, _ = np.linalg.qr(s.stream(191, 1).standard_normal((m, m)))
        Wu, _, Hu = o.rhals_sweep(U, U.T @ X, W, U.T @ W, H, order=order, reg=r)
        assert np.allclose(Wu, Wh, atol=1e-11) and np.allclose(Hu, Hh, atol=1e-11)


def test_regularized_rhals_w_step_is_the_printed_rule_on_the_surrogate():
    # One W column of the compressed sweep equals the printed regularized W
    # rule applied to X^ = Q B with W = Q W~ (Sec. 3.4 substituted as in R19).
    r = REGS["elastic"]
    X = s.low_rank_rows(30, 24, 4, 201, noise_abs=0.05)
    Q = o.range_finder(X, s.omega(24, 8, 201), 1)
    B = Q.T @ X
    W, H = s.init_factors(30, 24, 3, 201)
    Wt = Q.T @ W
    Wn, Wtn, Hn = o.rhals_sweep(Q, B, W, Wt, H, order=o.ORDER_W_FIRST, reg=r)
    # replay column by column in the high-dimensional frame
    V = H @ H.T
    Xh = Q @ B
    Wf = Q @ Wt
    Wt2 = Wt.copy()
    for j in range(3):
        v = V[j, j]
        d = v + r.alpha_w
        z = (v * Wf[:, j] + Xh @ H[j] - r.beta_w - Wf @ V[:, j]) / d
        col = np.where(z > 0, z, 0.0)
        Wt2[:, j] = Q.T @ col
        Wf[:, j] = Q @ Wt2[:, j]
        assert np.allclose(col, Wn[:, j], atol=1e-12)
    assert np.allclose(Wt2, Wtn, atol=1e-12)


def test_large_lasso_weight_zeroes_the_factor():
    # Sec. 3.4: the 1-norm promotes sparsity; past the largest possible
    # numerator every H row update is clipped to zero.
    X = s.low_rank_rows(20, 16, 3, 211, noise_abs=0.05)
    W, H = s.init_factors(20, 16, 3, 211)
    big = 10.0 * (np.abs(X.T @ W).max() + np.abs(W.T @ W).max() * np.abs(H).max() * 3 + 1.0)
    _, Hn = o.hals_sweep(X, W, H, o.ORDER_H_FIRST, reg=o.Reg(beta_h=big))
    assert np.all(Hn == 0.0)
    # and a moderate weight gives more zeros than none
    Wa, Ha, _ = o.hals(X, W, H, max_iter=200)
    Wb, Hb, _ = o.hals(X, W, H, max_iter=200, reg=o.Reg(beta_h=0.5, beta_w=0.5))
    assert np.count_nonzero(Hb == 0) + np.count_nonzero(Wb == 0) > np.count_nonzero(Ha == 0) + np.count_nonzero(Wa == 0)
