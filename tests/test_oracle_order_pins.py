"""Pins for the update orders of the oracle (Sec. 3.2: the interleaved and the
blocked cyclic orders and the shuffled order; reading R24): the ordered
sweeps with a blocked list reproduce the phase sweeps; every block update of
an interleaved or shuffled list is the explicit minimiser of its block
(scipy's NNLS and LAPACK least squares); a shuffled blocked order matches
scikit-learn's shuffled coordinate descent; the identity basis reduces the
compressed sweep to the deterministic one; the deterministic objective never
increases; exact low rank is recovered in any order."""

import warnings

import numpy as np
import pytest

import oracle as o
import synth as s

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def _nnls_1col(w, R):
    # argmin_{h >= 0} ||R - w h^T||_F, column by column, by scipy's NNLS.
    from scipy.optimize import nnls
    A = w.reshape(-1, 1)
    return np.array([nnls(A, R[:, c])[0][0] for c in range(R.shape[1])])


def _setup(seed, m=30, n=24, k=4, l=9):
    X = s.low_rank_rows(m, n, 5, seed, noise_abs=0.05)
    Q = o.range_finder(X, s.omega(n, l, seed), 1)
    W0, H0 = s.init_factors(m, n, k, seed)
    return X, Q, Q.T @ X, W0, Q.T @ W0, H0


def _shuffled(k, seed):
    return o.order_interleaved(k, s.stream(seed, 55).permutation(k))


def test_orders_use_every_block_once():
    k = 5
    for order in (o.order_blocked(k), o.order_blocked(k, True), o.order_interleaved(k), _shuffled(k, 3)):
        assert sorted(order) == list(range(2 * k))
    assert o.order_interleaved(3) == [0, 3, 1, 4, 2, 5]
    assert o.order_blocked(3) == [3, 4, 5, 0, 1, 2]


@pytest.mark.parametrize("w_first", [False, True])
def test_blocked_lists_reproduce_the_phase_sweeps(w_first):
    X, Q, B, W, Wt, H = _setup(301)
    k = H.shape[0]
    order = o.ORDER_W_FIRST if w_first else o.ORDER_H_FIRST
    a = o.rhals_sweep(Q, B, W, Wt, H, order=order)
    b = o.rhals_sweep_ordered(Q, B, W, Wt, H, o.order_blocked(k, w_first))
    for u, v in zip(a, b):
        assert np.allclose(u, v, rtol=1e-12, atol=1e-13)
    c = o.hals_sweep(X, W, H, order)
    d = o.hals_sweep_ordered(X, W, H, o.order_blocked(k, w_first))
    for u, v in zip(c, d):
        assert np.allclose(u, v, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("kind", ["interleaved", "shuffled"])
def test_ordered_block_updates_are_explicit_minimisers(kind):
    # Deterministic: each block is the NNLS minimiser of the explicit residual.
    # Compressed: H rows are the NNLS minimisers on X^ = Q B with the true W;
    # W~ columns the unconstrained minimisers of the compressed residual,
    # then lift, clip and map back (Sec. 3.2).
    X, Q, B, W, Wt, H = _setup(302)
    k = H.shape[0]
    order = o.order_interleaved(k) if kind == "interleaved" else _shuffled(k, 302)
    Wd, Hd = o.hals_sweep_ordered(X, W, H, order)
    Wr, Wtr, Hr = o.rhals_sweep_ordered(Q, B, W, Wt, H, order)
    Wb, Hb = W.copy(), H.copy()
    Wc, Wtc, Hc = W.copy(), Wt.copy(), H.copy()
    Xh = Q @ B
    for e in order:
        if e < k:
            j = e
            Rj = X - Wb @ Hb + np.outer(Wb[:, j], Hb[j, :])
            Wb[:, j] = _nnls_1col(Hb[j, :], Rj.T)
            Rt = B - Wtc @ Hc + np.outer(Wtc[:, j], Hc[j, :])
            w, *_ = np.linalg.lstsq(Hc[j, :].reshape(-1, 1), Rt.T, rcond=None)
            Wc[:, j] = np.maximum(Q @ w.ravel(), 0.0)
            Wtc[:, j] = Q.T @ Wc[:, j]
        else:
            j = e - k
            Rj = X - Wb @ Hb + np.outer(Wb[:, j], Hb[j, :])
            Hb[j, :] = _nnls_1col(Wb[:, j], Rj)
            Rh = Xh - Wc @ Hc + np.outer(Wc[:, j], Hc[j, :])
            Hc[j, :] = _nnls_1col(Wc[:, j], Rh)
    assert np.allclose(Wd, Wb, atol=1e-10) and np.allclose(Hd, Hb, atol=1e-10)
    assert np.allclose(Wr, Wc, atol=1e-10) and np.allclose(Hr, Hc, atol=1e-10)
    assert np.allclose(Wtr, Wtc, atol=1e-10)


def test_shuffled_blocked_order_matches_scikit_learn():
    # scikit-learn's coordinate descent with shuffle draws one permutation of
    # the W columns, then one of the H rows, per iteration, from one
    # RandomState; the same lists give the same iterates.
    nmf = pytest.importorskip("sklearn.decomposition._nmf")
    m, n, k, iters, seed = 30, 25, 5, 12, 7
    g = s.stream(311, 99)
    X, W0, H0 = g.random((m, n)), g.random((m, k)), g.random((k, n))
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        Ws, Hs, it = nmf._fit_coordinate_descent(X, W0.copy(), H0.copy(), tol=0.0, max_iter=iters,
                                                  shuffle=True, random_state=seed)
    rs = np.random.RandomState(seed)
    W, H = W0, H0
    for _ in range(iters):
        pw = rs.permutation(k)
        ph = rs.permutation(k)
        W, H = o.hals_sweep_ordered(X, W, H, [int(j) for j in pw] + [k + int(j) for j in ph])
    assert it == iters
    assert np.allclose(W, Ws, rtol=1e-10, atol=1e-12) and np.allclose(H, Hs, rtol=1e-10, atol=1e-12)


def test_identity_basis_reduces_ordered_rhals_to_ordered_hals():
    m, n, k = 12, 30, 3
    X = s.stream(312, 99).random((m, n))
    W, H = s.init_factors(m, n, k, 312)
    for order in (o.order_interleaved(k), _shuffled(k, 312)):
        Wh, Hh = o.hals_sweep_ordered(X, W, H, order)
        Wr, _, Hr = o.rhals_sweep_ordered(np.eye(m), X, W, W.copy(), H, order)
        assert np.array_equal(Wh, Wr) and np.array_equal(Hh, Hr)


def test_ordered_hals_objective_is_monotone():
    X = s.low_rank_rows(40, 30, 5, 313, noise_abs=0.05)
    W, H = s.init_factors(40, 30, 4, 313)
    for kind in ("interleaved", "shuffled"):
        Wc, Hc = W.copy(), H.copy()
        fc = np.linalg.norm(X - Wc @ Hc) ** 2
        for it in range(60):
            order = o.order_interleaved(4) if kind == "interleaved" else _shuffled(4, 1000 + it)
            Wc, Hc = o.hals_sweep_ordered(X, Wc, Hc, order)
            fn = np.linalg.norm(X - Wc @ Hc) ** 2
            assert fn <= fc * (1 + 1e-12)
            fc = fn


@pytest.mark.parametrize("kind", ["interleaved", "shuffled"])
def test_exact_low_rank_is_recovered_in_any_order(kind):
    m, n, r = 60, 50, 3
    g = s.stream(1002, 0)
    X = g.random((m, r)) @ g.random((r, n))
    W, H = s.init_factors(m, n, r, 2002)
    Q = o.range_finder(X, s.omega(n, r + 5, 3002), 1)
    B = Q.T @ X
    Wd, Hd = W.copy(), H.copy()
    Wr, Wtr, Hr = W.copy(), Q.T @ W, H.copy()
    for it in range(3000):
        order = o.order_interleaved(r) if kind == "interleaved" else _shuffled(r, 5000 + it)
        Wd, Hd = o.hals_sweep_ordered(X, Wd, Hd, order)
        Wr, Wtr, Hr = o.rhals_sweep_ordered(Q, B, Wr, Wtr, Hr, order)
    # the orders converge at different rates on this instance (after 3000
    # sweeps: interleaved 1e-13 and 5e-16, shuffled 2e-10 and 1e-9)
    bar = 1e-10 if kind == "interleaved" else 1e-8
    assert o.rel_error(X, Wd, Hd) <= bar
    assert o.rel_error(X, Wr, Hr) <= bar
