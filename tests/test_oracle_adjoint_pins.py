"""Pins for the reference gradients of unrolled randomized-HALS sweeps
(oracle/adjoint.py; readings R21-R23): the torch transcription reproduces the
NumPy oracle's sweeps, and its reverse-mode derivatives agree with central
finite differences along random directions at points where a step of +-h
leaves every clip decision unchanged."""

import numpy as np
import pytest

import oracle as o
import synth as s

torch = pytest.importorskip("torch")
from oracle import adjoint as A  # noqa: E402


def _setup(m, n, k, l, seed, T):
    X = s.low_rank_rows(m, n, k + 2, seed, noise_abs=0.02)
    Q = o.range_finder(X, s.omega(n, l, seed), 1)
    W0, H0 = s.init_factors(m, n, k, seed)
    return X, Q, W0, H0


def test_torch_transcription_reproduces_the_oracle_sweeps():
    X, Q, W0, H0 = _setup(60, 45, 4, 9, 501, 4)
    B = Q.T @ X
    W, Wt, H = W0, Q.T @ W0, H0
    for _ in range(4):
        W, Wt, H = o.rhals_sweep(Q, B, W, Wt, H)
    Wt_, Ht_ = A.unrolled(torch.tensor(Q), torch.tensor(X), torch.tensor(W0), torch.tensor(H0), 4)
    assert np.allclose(Wt_.numpy(), W, atol=1e-12) and np.allclose(Ht_.numpy(), H, atol=1e-12)


def _loss_np(Q, X, W0, H0, T):
    with torch.no_grad():
        W, H = A.unrolled(torch.tensor(Q), torch.tensor(X), torch.tensor(W0), torch.tensor(H0), T)
        return float(A.loss_t(torch.tensor(X), W, H))


@pytest.mark.parametrize("m,n,k,l,T,seed", [(40, 30, 3, 6, 3, 502), (256, 128, 8, 16, 5, 503)])
def test_gradients_match_central_differences(m, n, k, l, T, seed):
    X, Q, W0, H0 = _setup(m, n, k, l, seed, T)
    gX, gW0, gH0, L, _, _ = A.grads(Q, X, W0, H0, T)
    rng = s.stream(seed, 77)
    h = 1e-6
    base = A.active_sets(Q, X, W0, H0, T)
    checked = 0
    for trial in range(6):
        dX = rng.standard_normal(X.shape)
        dW = rng.standard_normal(W0.shape)
        dH = rng.standard_normal(H0.shape)
        plus = (X + h * dX, W0 + h * dW, H0 + h * dH)
        minus = (X - h * dX, W0 - h * dW, H0 - h * dH)
        same = all(all(np.array_equal(a, b) for a, b in zip(base, A.active_sets(Q, *pt, T))) for pt in (plus, minus))
        if not same:
            continue  # a clip decision flips within +-h: the derivative is not defined there
        fd = (_loss_np(Q, *plus, T) - _loss_np(Q, *minus, T)) / (2 * h)
        an = float(np.sum(gX * dX) + np.sum(gW0 * dW) + np.sum(gH0 * dH))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (trial, fd, an)
        checked += 1
    assert checked >= 3


def test_upstream_gradient_form_is_the_vector_jacobian_product():
    # with upstream gradients (gW, gH) the reference returns <gW, dW_T> + <gH, dH_T>
    # derivatives; X enters through B only
    X, Q, W0, H0 = _setup(50, 40, 3, 7, 504, 3)
    rng = s.stream(504, 78)
    gW, gH = rng.standard_normal((50, 3)), rng.standard_normal((3, 40))
    gX, gW0, gH0, _, WT, HT = A.grads(Q, X, W0, H0, 3, gW, gH)
    h = 1e-6
    dX, dW, dH = rng.standard_normal(X.shape), rng.standard_normal(W0.shape), rng.standard_normal(H0.shape)

    def f(Xp, Wp, Hp):
        with torch.no_grad():
            W, H = A.unrolled(torch.tensor(Q), torch.tensor(Xp), torch.tensor(Wp), torch.tensor(Hp), 3)
        return float(np.sum(W.numpy() * gW) + np.sum(H.numpy() * gH))

    fd = (f(X + h * dX, W0 + h * dW, H0 + h * dH) - f(X - h * dX, W0 - h * dW, H0 - h * dH)) / (2 * h)
    an = float(np.sum(gX * dX) + np.sum(gW0 * dW) + np.sum(gH0 * dH))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    # dB = Q^T dX: the X gradient lies in the range of Q
    assert np.linalg.norm(gX - Q @ (Q.T @ gX)) <= 1e-10 * np.linalg.norm(gX)


def test_clipped_entries_pass_no_gradient():
    # an H entry clipped to zero in the last sweep has zero derivative of H_T
    # with respect to anything upstream of its own clip (reading R22)
    X, Q, W0, H0 = _setup(30, 25, 3, 6, 505, 1)
    _, _, _, _, WT, HT = A.grads(Q, X, W0, H0, 1)
    zero = np.argwhere(HT == 0.0)
    if len(zero) == 0:
        pytest.skip("no clipped entry in this draw")
    j, c = zero[0]
    gH = np.zeros_like(HT)
    gH[j, c] = 1.0
    gX, gW0, gH0, _, _, _ = A.grads(Q, X, W0, H0, 1, np.zeros_like(WT), gH)
    assert np.all(gX == 0.0) and np.all(gW0 == 0.0) and np.all(gH0 == 0.0)


def _setup_clipping(m, n, k, l, seed, rank, noise):
    # rank below k and strong noise: many entries of W and H are clipped
    X = s.low_rank_rows(m, n, rank, seed, noise_abs=noise)
    Q = o.range_finder(X, s.omega(n, l, seed), 1)
    W0, H0 = s.init_factors(m, n, k, seed)
    return X, Q, W0, H0


@pytest.mark.parametrize("m,n,k,l,T,seed,rank,noise", [(40, 30, 4, 8, 3, 502, 2, 0.05),
                                                       (120, 90, 6, 12, 4, 504, 3, 0.2)])
def test_masked_gradients_equal_the_clipped_ones_on_the_own_trajectory(m, n, k, l, T, seed, rank, noise):
    # with the activities of the float64 trajectory itself, the masked sweeps
    # are the same map on the same piece: identical loss and gradients
    X, Q, W0, H0 = _setup_clipping(m, n, k, l, seed, rank, noise)
    gX, gW0, gH0, L, _, _ = A.grads(Q, X, W0, H0, T)
    masks = A.trajectory_masks(Q, X, W0, H0, T)
    assert any(not mW.all() for mW, _ in masks) and any(not mH.all() for _, mH in masks)  # clips are active
    mX, mW0, mH0, mL = A.grads_masked(Q, X, W0, H0, T, masks)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert abs(mL - L) <= 1e-12 * abs(L)
    assert rel(mX, gX) <= 1e-12 and rel(mW0, gW0) <= 1e-12 and rel(mH0, gH0) <= 1e-12


def test_masked_gradients_follow_the_given_activities():
    # a flipped activity changes the piece: the loss and the gradient move
    X, Q, W0, H0 = _setup_clipping(40, 30, 4, 8, 505, 2, 0.05)
    masks = A.trajectory_masks(Q, X, W0, H0, 3)
    mW, mH = masks[0]
    flipped = [(mW.copy(), mH.copy())] + masks[1:]
    i, j = np.argwhere(mH)[0]
    flipped[0][1][i, j] = False
    g0 = A.grads_masked(Q, X, W0, H0, 3, masks)
    g1 = A.grads_masked(Q, X, W0, H0, 3, flipped)
    assert not np.allclose(g0[2], g1[2], rtol=1e-9, atol=0)
