"""Reference gradients of unrolled randomized-HALS sweeps, float64, by automatic
differentiation of a literal torch transcription of the sweep.

Test infrastructure only (see the package docstring).

The method being differentiated is Algorithm 1's sweep (Sec. 3.2) with the
basis Q held fixed: GRAM_FULL (S = W^T W), H rows first, then W columns with
lift, clip and map-back, exactly as :func:`oracle.rhals.rhals_sweep`.  The
paper does not differentiate the method; the readings are:

R21 Q is a constant of the unrolled map (the range finder is not
    differentiated), B = Q^T X, and W~0 = Q^T W0.
R22 The derivative of max(0, x) is taken as 0 at x = 0 (and 1 for x > 0).
    Every block update is written as the paper prints it, so a row or column
    that is replaced has no derivative with respect to its own old value
    (the two terms cancel exactly).
R23 The loss used for checks is ||X - W H||_F^2 + sum(H) (H >= 0, so the
    1-norm is the sum).  Its direct terms are left to the caller; the
    unrolled map returns (W_T, H_T).
"""

import numpy as np

try:  # torch is the differentiation engine for the reference only
    import torch
except ImportError:  # pragma: no cover - torch is installed where tests run
    torch = None


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def rhals_sweep_t(Q, B, W, Wt, H):
    """One sweep of Algorithm 1 in torch float64 (GRAM_FULL, H rows first),
    written without in-place updates so that autograd can follow it.  Blocks
    with a zero scale are skipped (reading R9)."""
    k = H.shape[0]
    # H phase: R = B^T W~, S = W^T W, rows of H in turn
    R = B.T @ Wt
    S = W.T @ W
    rows = [H[j] for j in range(k)]
    for j in range(k):
        d = S[j, j]
        if d.item() > 0.0:
            Hc = torch.stack(rows)
            a = rows[j] + (R[:, j] - Hc.T @ S[:, j]) / d
            rows[j] = torch.clamp(a, min=0.0)
    H = torch.stack(rows)
    # W phase: T = B H^T, V = H H^T, columns of W~ in turn
    T = B @ H.T
    V = H @ H.T
    wt_cols = [Wt[:, j] for j in range(k)]
    w_cols = [W[:, j] for j in range(k)]
    for j in range(k):
        d = V[j, j]
        if d.item() > 0.0:
            Wtc = torch.stack(wt_cols, dim=1)
            u = wt_cols[j] + (T[:, j] - Wtc @ V[:, j]) / d
            w = torch.clamp(Q @ u, min=0.0)
            w_cols[j] = w
            wt_cols[j] = Q.T @ w
    return torch.stack(w_cols, dim=1), torch.stack(wt_cols, dim=1), H


def rhals_sweep_t_masked(Q, B, W, Wt, H, mW, mH):
    """rhals_sweep_t with every clip replaced by a given activity: mH (k x n)
    and mW (m x k) hold 1 where the clipped value is kept and 0 where it is
    set to zero.  With the activities of a trajectory, this sweep is the
    linear piece of the unrolled map that the trajectory lies on; its
    derivative is the one reading R22 gives there (0 where the activity is
    0, including a pre-clip value of exactly 0)."""
    k = H.shape[0]
    R = B.T @ Wt
    S = W.T @ W
    rows = [H[j] for j in range(k)]
    for j in range(k):
        d = S[j, j]
        if d.item() > 0.0:
            Hc = torch.stack(rows)
            a = rows[j] + (R[:, j] - Hc.T @ S[:, j]) / d
            rows[j] = a * mH[j]
    H = torch.stack(rows)
    T = B @ H.T
    V = H @ H.T
    wt_cols = [Wt[:, j] for j in range(k)]
    w_cols = [W[:, j] for j in range(k)]
    for j in range(k):
        d = V[j, j]
        if d.item() > 0.0:
            Wtc = torch.stack(wt_cols, dim=1)
            u = wt_cols[j] + (T[:, j] - Wtc @ V[:, j]) / d
            w = (Q @ u) * mW[:, j]
            w_cols[j] = w
            wt_cols[j] = Q.T @ w
    return torch.stack(w_cols, dim=1), torch.stack(wt_cols, dim=1), H


def unrolled(Q, X, W0, H0, T):
    """(W_T, H_T) after T sweeps from W0, H0 on B = Q^T X (reading R21), as
    torch float64 tensors connected to X, W0 and H0."""
    B = Q.T @ X
    W, Wt, H = W0, Q.T @ W0, H0
    for _ in range(T):
        W, Wt, H = rhals_sweep_t(Q, B, W, Wt, H)
    return W, H


def loss_t(X, W, H):
    """||X - W H||_F^2 + sum(H) (reading R23)."""
    E = X - W @ H
    return (E * E).sum() + H.sum()


def grads(Q, X, W0, H0, T, gW=None, gH=None):
    """Reverse-mode gradients through T unrolled sweeps.

    With gW, gH (upstream gradients of W_T, H_T) given: returns
    (gX, gW0, gH0) of <gW, W_T> + <gH, H_T> (X enters through B = Q^T X only).
    Without them: the gradients of the loss of reading R23 (X enters through
    B and directly).  Returns numpy float64 arrays and the loss value."""
    if torch is None:
        raise RuntimeError("torch is needed for the reference gradients")
    Qt = _t(Q)
    Xt = _t(X).requires_grad_(True)
    W0t = _t(W0).requires_grad_(True)
    H0t = _t(H0).requires_grad_(True)
    W, H = unrolled(Qt, Xt, W0t, H0t, T)
    if gW is None:
        L = loss_t(Xt, W, H)
    else:
        L = (W * _t(gW)).sum() + (H * _t(gH)).sum()
    L.backward()
    return (Xt.grad.numpy(), W0t.grad.numpy(), H0t.grad.numpy(), float(L.detach()),
            W.detach().numpy(), H.detach().numpy())


def trajectory_masks(Q, X, W0, H0, T):
    """Activities (W_t > 0, H_t > 0) after each of the T sweeps of the float64
    trajectory, as boolean numpy arrays."""
    if torch is None:
        raise RuntimeError("torch is needed for the reference gradients")
    Qt, B = _t(Q), _t(Q).T @ _t(X)
    W, Wt, H = _t(W0), _t(Q).T @ _t(W0), _t(H0)
    out = []
    with torch.no_grad():
        for _ in range(T):
            W, Wt, H = rhals_sweep_t(Qt, B, W, Wt, H)
            out.append(((W > 0).numpy().copy(), (H > 0).numpy().copy()))
    return out


def grads_masked(Q, X, W0, H0, T, masks):
    """Gradients of the loss of reading R23 through T sweeps in which sweep t
    uses the activities masks[t] = (mW, mH) instead of its clips: the
    derivative of the unrolled map on the piece those activities select.
    Given the activities of a trajectory computed in another precision, it
    is that trajectory's exact gradient, free of the clip decisions that
    rounding moved.  Returns (gX, gW0, gH0, loss)."""
    if torch is None:
        raise RuntimeError("torch is needed for the reference gradients")
    Qt = _t(Q)
    Xt = _t(X).requires_grad_(True)
    W0t = _t(W0).requires_grad_(True)
    H0t = _t(H0).requires_grad_(True)
    B = Qt.T @ Xt
    W, Wt, H = W0t, Qt.T @ W0t, H0t
    for t in range(T):
        mW, mH = masks[t]
        W, Wt, H = rhals_sweep_t_masked(Qt, B, W, Wt, H, _t(mW), _t(mH))
    L = loss_t(Xt, W, H)
    L.backward()
    return Xt.grad.numpy(), W0t.grad.numpy(), H0t.grad.numpy(), float(L.detach())


def active_sets(Q, X, W0, H0, T):
    """Signs of every pre-clip value along the unrolled map, for checking that
    a finite-difference step leaves the active set unchanged."""
    Qt, B = _t(Q), _t(Q).T @ _t(X)
    W, Wt, H = _t(W0), _t(Q).T @ _t(W0), _t(H0)
    signs = []
    k = H.shape[0]
    for _ in range(T):
        R = B.T @ Wt
        S = W.T @ W
        rows = [H[j] for j in range(k)]
        for j in range(k):
            if S[j, j].item() > 0.0:
                Hc = torch.stack(rows)
                a = rows[j] + (R[:, j] - Hc.T @ S[:, j]) / S[j, j]
                signs.append((a > 0).numpy().copy())
                rows[j] = torch.clamp(a, min=0.0)
        H = torch.stack(rows)
        Tm, V = B @ H.T, H @ H.T
        wt_cols = [Wt[:, j] for j in range(k)]
        w_cols = [W[:, j] for j in range(k)]
        for j in range(k):
            if V[j, j].item() > 0.0:
                Wtc = torch.stack(wt_cols, dim=1)
                u = wt_cols[j] + (Tm[:, j] - Wtc @ V[:, j]) / V[j, j]
                z = Qt @ u
                signs.append((z > 0).numpy().copy())
                w_cols[j] = torch.clamp(z, min=0.0)
                wt_cols[j] = Qt.T @ w_cols[j]
        W, Wt = torch.stack(w_cols, dim=1), torch.stack(wt_cols, dim=1)
    return signs
