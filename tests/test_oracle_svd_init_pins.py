"""Pins for the SVD-based initialization of the oracle (the Remark on
initialization after Algorithm 1; reading R20): the nonnegative double SVD of
the randomized SVD from the QB decomposition.  Each check rests on something
outside the oracle's own formula: scikit-learn's implementation of the same
published scheme, LAPACK's SVD (best rank-one approximations, the Perron
pair), and invariances of the singular value decomposition."""

import numpy as np
import pytest

import oracle as o
import synth as s


def _exact_rank(m, n, r, seed):
    g = s.stream(seed, 0)
    return g.random((m, r)) @ g.random((r, n))


def test_svd_init_matches_scikit_learn_nndsvd_on_exact_low_rank_data():
    # With X of rank k the randomized SVD from Q B is exact, so it must agree
    # with scikit-learn's NNDSVD of X (its own randomized SVD is exact too).
    nmf = pytest.importorskip("sklearn.decomposition._nmf")
    m, n, k = 60, 45, 5
    X = _exact_rank(m, n, k, 401)
    Q = o.range_finder(X, s.omega(n, k + 4, 401), 2)
    W, H = o.svd_init(Q, Q.T @ X, k)
    Ws, Hs = nmf._initialize_nmf(X, k, init="nndsvd", eps=0.0, random_state=0)
    assert np.allclose(W, Ws, atol=1e-9) and np.allclose(H, Hs, atol=1e-9)


def test_each_component_is_the_best_rank_one_fit_of_the_positive_section():
    # Boutsidis and Gallopoulos: the positive section max(0, s_j u_j v_j^T) of
    # a rank-one term is x+ y+^T + x- y-^T (disjoint supports), and the
    # component keeps the dominant term, i.e. its best rank-one approximation.
    X = s.low_rank_rows(50, 40, 6, 402, noise_abs=0.05)
    Q = o.range_finder(X, s.omega(40, 12, 402), 1)
    B = Q.T @ X
    k = 6
    W, H = o.svd_init(Q, B, k)
    Ub, sv, Vt = np.linalg.svd(B, full_matrices=False)
    U = Q @ Ub
    for j in range(1, k):
        C = np.maximum(sv[j] * np.outer(U[:, j], Vt[j]), 0.0)
        a, b, c = np.linalg.svd(C)
        best = b[0] * np.outer(a[:, 0], c[0])
        assert np.allclose(np.outer(W[:, j], H[j]), best, atol=1e-10 * max(1.0, b[0]))
    assert W.min() >= 0.0 and H.min() >= 0.0


def test_leading_component_is_the_perron_pair():
    # for nonnegative X the leading singular vectors are single-signed, so
    # W_1 H_1 is the best rank-one approximation of X^ = Q B
    X = s.low_rank_rows(40, 30, 4, 403, noise_abs=0.02)
    Q = o.range_finder(X, s.omega(30, 8, 403), 2)
    B = Q.T @ X
    W, H = o.svd_init(Q, B, 3)
    a, b, c = np.linalg.svd(Q @ B)
    assert np.allclose(np.outer(W[:, 0], H[0]), b[0] * np.outer(a[:, 0], c[0]), atol=1e-10 * b[0])


def test_nndsvd_is_invariant_to_singular_vector_signs():
    X = s.low_rank_rows(30, 25, 5, 404, noise_abs=0.05)
    U, sv, Vt = np.linalg.svd(X, full_matrices=False)
    W, H = o.nndsvd(U[:, :5], sv[:5], Vt[:5])
    flip = np.array([1.0, -1.0, -1.0, 1.0, -1.0])
    W2, H2 = o.nndsvd(U[:, :5] * flip, sv[:5], Vt[:5] * flip[:, None])
    assert np.array_equal(W, W2) and np.array_equal(H, H2)


def test_svd_init_does_not_depend_on_the_basis_rotation():
    # Q -> Q R with R orthogonal (l x l) leaves Q B and hence the init unchanged
    X = s.low_rank_rows(40, 30, 6, 405, noise_abs=0.05)
    Q = o.range_finder(X, s.omega(30, 9, 405), 1)
    B = Q.T @ X
    R, _ = np.linalg.qr(s.stream(405, 1).standard_normal((9, 9)))
    W, H = o.svd_init(Q, B, 4)
    W2, H2 = o.svd_init(Q @ R, R.T @ B, 4)
    assert np.allclose(W, W2, atol=1e-10) and np.allclose(H, H2, atol=1e-10)


def test_degenerate_component_is_zero():
    # x entirely nonnegative and y entirely nonpositive: both products vanish
    U = np.array([[1.0, 0.6], [0.0, 0.8]])
    Vt = np.array([[1.0, 0.0], [-0.6, -0.8]])
    W, H = o.nndsvd(U, np.array([2.0, 1.0]), Vt)
    assert np.all(W[:, 1] == 0.0) and np.all(H[1] == 0.0)
    assert np.allclose(W[:, 0], np.sqrt(2.0) * np.array([1.0, 0.0]))
