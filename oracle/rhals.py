"""Deterministic and randomized HALS for NMF, float64, written from the paper.

Test infrastructure only (see the package docstring).

Source: Erichson et al., "Randomized Nonnegative Matrix Factorization",
arXiv:1711.02037.

* Sec. 2.1, Eq. (lowrank) and Sec. 2.2, Eq. (nmf_opt): the problem, X ~ W H with
  W, H >= 0 minimising ||X - W H||_F^2.
* Sec. 2.3: the randomized QB decomposition (sketch, oversampling, subspace
  iteration, QR, B = Q^T X) and Appendix A, Algorithm 2 (column-streamed QB).
* Sec. 3.1: HALS block updates and their residual-free form.
* Sec. 3.2 and Algorithm 1: randomized HALS on the compressed matrix B.
* Sec. 3.3: the projected-gradient stopping rule.

Readings taken where the paper is silent, ambiguous or misprinted (each is also
listed in the design document):

R1  Sketch width l = min(k + p, min(m, n)).
R2  The QR factor is the thin QR with a nonnegative diagonal of R, which makes
    Q unique for full-rank input (the paper does not fix the sign convention).
R3  Subspace iteration follows Algorithm 1 (re-orthonormalise after each
    half-step), not the fused power step of Algorithm 2.
R4  The compressed factor starts as W~ = Q^T W0 (Algorithm 1 only says that
    W, W~ and H are initialised).
R5  Default order inside a sweep is Algorithm 1's: all rows of H, then all
    columns of W.  The other blocked order (all columns of W first, which
    Sec. 3.2 says it prefers) is ORDER_W_FIRST.
R6  Default Gram in the H update is S = W^T W (Algorithm 1).  GRAM_LOWDIM uses
    W~^T W~ for numerator and denominator (the H rule printed in Sec. 3.2);
    GRAM_MIXED uses W~^T W~ in the numerator and (W^T W)_jj as the scale, as
    the note after that rule suggests.
R7  The lift in Algorithm 1 is read as W(:,j) = max(0, Q W~(:,j)) (the
    algorithm box misprints W for W~; Sec. 3.2 gives the lift).
R8  Printed sizes are read as Omega: n x l, Q: m x l, B: l x n, T: l x k.
R9  A block whose scale is exactly zero (S_jj = 0 or V_jj = 0) is skipped; for
    the W step this skips the update, the lift and the map-back.
R10 The projected gradient of Sec. 3.3 is evaluated after each full sweep, with
    the factor 2 dropped (it cancels in the ratio).  For randomized HALS it is
    taken on the surrogate X^ = Q B.
R11 "Relative error" is ||X - W H||_F / ||X||_F, computed directly.
R12 max(0, x) is computed as (x if x > 0 else +0).
R24 Update orders (Sec. 3.2): besides the two blocked orders, the interleaved
    order W(:,1) -> H(1,:) -> ... -> W(:,k) -> H(k,:) and the shuffled order,
    read as the interleaved order over a random permutation of the components
    per sweep (the permutation is an input).  Each block update takes the
    products of the factors as they are at that moment.
R18 Regularized rules (Sec. 3.4 and its appendix) are taken as printed: the
    ridge weight alpha enlarges the scale (S_jj + alpha, V_jj + alpha) and
    damps the old block by S_jj / (S_jj + alpha); the LASSO weight beta is
    subtracted from the cross product.  These are the exact block minimisers of
    1/2 ||X - W H||_F^2 + alpha/2 ||F||_F^2 + beta sum(F) over F >= 0, so the
    projected gradient of Sec. 3.3 gains + alpha F + beta (factor 2 dropped as
    in R10).  The H rule's misprinted W^T W~ in the first scale is read as the
    scale used everywhere else.  The elastic net (the two combined) keeps
    these letters: alpha for the squared norm, beta for the 1-norm.
R19 In randomized HALS the ridge part acts on W~ (it is linear) while the
    LASSO shift beta / (V_jj + alpha) is applied to the lifted column before
    the clip: substituting X ~ Q B and W ~ Q W~ into the printed W rule leaves
    the all-ones m-vector outside the range of Q.  With Q square and
    orthogonal the sweep is the deterministic regularized sweep.
R20 SVD-based initialization (the Remark on initialization after Algorithm 1
    points to the nonnegative double SVD of Boutsidis and Gallopoulos, 2008)
    is taken on the randomized SVD of the QB decomposition: B = U_B S V^T,
    U = Q U_B.  Component 1 takes |u_1|, |v_1|; every other component keeps
    the positive or the negative parts of (u_j, v_j), whichever has the
    larger product of norms (ties go to the negative parts), scaled by
    sqrt(s_j * that product).  A component whose two products are both zero
    is set to zero.  Zero entries stay zero (no fill).
"""

from typing import NamedTuple

import numpy as np

GRAM_FULL = 0     # S = W^T W           (Algorithm 1)
GRAM_LOWDIM = 1   # S = W~^T W~         (Sec. 3.2, H rule as printed)
GRAM_MIXED = 2    # numerator W~^T W~, scale (W^T W)_jj (Sec. 3.2, note)

ORDER_H_FIRST = 0  # Algorithm 1: rows of H, then columns of W
ORDER_W_FIRST = 1  # Sec. 3.2, second cyclic order: columns of W, then rows of H


class Reg(NamedTuple):
    """Regularization weights of Sec. 3.4 (reading R18): alpha_* for the
    squared Frobenius norm (ridge), beta_* for the 1-norm (LASSO); both
    nonzero is the elastic net.  All zero is plain HALS."""
    alpha_w: float = 0.0
    alpha_h: float = 0.0
    beta_w: float = 0.0
    beta_h: float = 0.0


NO_REG = Reg()


def clip(x):
    """[x]_+ = max(0, x) elementwise (Sec. 3.1, after the HALS rules); reading R12."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > 0.0, x, 0.0)


def sketch_width(k, p, m, n):
    """Oversampled sketch width l = k + p (Algorithm 1; Sec. 2.3), clamped to
    min(m, n) (reading R1)."""
    return int(min(k + p, min(m, n)))


def qr_positive(Y):
    """Thin QR of a tall matrix by LAPACK Householder QR, with columns of Q
    scaled so that diag(R) >= 0 (reading R2).  Returns (Q, R)."""
    Y = np.asarray(Y, dtype=np.float64)
    Q, R = np.linalg.qr(Y, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def range_finder(X, Omega, q):
    """Orthonormal basis Q (m x l) of the approximate range of X.

    Sec. 2.3 (Eqs. YXC and AQQA, subspace iteration) and Algorithm 1 (sketch,
    q subspace iterations with a QR after each half-step, final QR).  Omega is
    the n x l test matrix, supplied by the caller.
    """
    X = np.asarray(X, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    Y = X @ Omega
    for _ in range(int(q)):
        Q, _ = qr_positive(Y)
        Qn, _ = qr_positive(X.T @ Q)
        Y = X @ Qn
    Q, _ = qr_positive(Y)
    return Q


def compress(X, Q):
    """B = Q^T X, the l x n surrogate (Sec. 2.3; Algorithm 1)."""
    return np.asarray(Q, dtype=np.float64).T @ np.asarray(X, dtype=np.float64)


def qb(X, Omega, q):
    """Randomized QB decomposition, Algorithm 1 form.  Returns (Q, B)."""
    Q = range_finder(X, Omega, q)
    return Q, compress(X, Q)


def qb_streaming(X, Omega, q, block=1):
    """Randomized QB decomposition in the column-streamed form of Appendix A,
    Algorithm 2: the sketch and the power step are accumulated one block of
    columns of X at a time, and B is formed column block by column block.

    The power step of that algorithm is read with the accumulator reset before
    each pass (the listing omits the reset and the accumulation).  It is used
    only as a cross-check of span(Q) on well-conditioned inputs.
    """
    X = np.asarray(X, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    m, n = X.shape
    l = Omega.shape[1]
    Y = np.zeros((m, l))
    for j0 in range(0, n, block):
        Y += X[:, j0:j0 + block] @ Omega[j0:j0 + block, :]
    for _ in range(int(q)):
        Q, _ = qr_positive(Y)
        Y = np.zeros((m, l))
        for j0 in range(0, n, block):
            A = X[:, j0:j0 + block]
            Y += A @ (A.T @ Q)
    Q, _ = qr_positive(Y)
    B = np.zeros((l, n))
    for j0 in range(0, n, block):
        B[:, j0:j0 + block] = Q.T @ X[:, j0:j0 + block]
    return Q, B


# ----------------------------------------------------------------------------
# SVD-based initialization (Remark on initialization; reading R20)
# ----------------------------------------------------------------------------

def nndsvd(U, sv, Vt):
    """Nonnegative double SVD (Boutsidis and Gallopoulos, 2008) of the
    singular triplets U (m x k), sv (k, descending), Vt (k x n): returns
    W (m x k) and H (k x n), both nonnegative (reading R20)."""
    U = np.asarray(U, dtype=np.float64)
    Vt = np.asarray(Vt, dtype=np.float64)
    sv = np.asarray(sv, dtype=np.float64)
    m, k = U.shape
    W = np.zeros((m, k))
    H = np.zeros((k, Vt.shape[1]))
    for j in range(k):
        x, y = U[:, j], Vt[j, :]
        if j == 0:
            W[:, 0] = np.sqrt(sv[0]) * np.abs(x)
            H[0, :] = np.sqrt(sv[0]) * np.abs(y)
            continue
        xp, xn = np.maximum(x, 0.0), np.maximum(-x, 0.0)
        yp, yn = np.maximum(y, 0.0), np.maximum(-y, 0.0)
        mp = np.linalg.norm(xp) * np.linalg.norm(yp)
        mn = np.linalg.norm(xn) * np.linalg.norm(yn)
        if mp > mn:
            u, v, sig = xp, yp, mp
        else:
            u, v, sig = xn, yn, mn
        if sig > 0.0:
            c = np.sqrt(sv[j] * sig)
            W[:, j] = c * u / np.linalg.norm(u)
            H[j, :] = c * v / np.linalg.norm(v)
    return W, H


def svd_init(Q, B, k):
    """W0, H0 from the randomized SVD of the QB decomposition (Sec. 2.3:
    X ~ Q B, B = U_B S V^T, so X ~ (Q U_B) S V^T) followed by the
    nonnegative double SVD of its k leading triplets (reading R20).  The SVD
    of the small l x n matrix B is LAPACK's."""
    Q = np.asarray(Q, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if not (1 <= k <= B.shape[0]):
        raise ValueError("need 1 <= k <= l")
    Ub, sv, Vt = np.linalg.svd(B, full_matrices=False)
    return nndsvd(Q @ Ub[:, :k], sv[:k], Vt[:k])


# ----------------------------------------------------------------------------
# Sweeps
# ----------------------------------------------------------------------------

def _h_rows(H, R, S_num, S_scale, alpha=0.0, beta=0.0):
    """Row-by-row H update, Gauss-Seidel over j (Algorithm 1; Sec. 3.1 and 3.2
    H rules, with the regularized form of Sec. 3.4):
    H(j,:) <- [s/(s+alpha) H(j,:) + (R(:,j) - beta - H^T S(:,j)) / (s+alpha)]_+
    with s = S_jj, the numerator Gram S_num and the scale S_scale (equal except
    in GRAM_MIXED).  Rows with zero scale s + alpha are skipped (reading R9).
    With alpha = beta = 0 this is the plain rule to the last bit."""
    k = H.shape[0]
    for j in range(k):
        s = S_scale[j, j]
        d = s + alpha
        if d > 0.0:
            H[j, :] = clip(s / d * H[j, :] + (R[:, j] - beta - H.T @ S_num[:, j]) / d)
    return H


def rhals_sweep(Q, B, W, Wt, H, gram_mode=GRAM_FULL, order=ORDER_H_FIRST, reg=NO_REG):
    """One sweep of randomized HALS (Algorithm 1; Sec. 3.2).

    Q: m x l orthonormal basis; B: l x n compressed data; W: m x k; Wt: the
    compressed factor W~ (l x k); H: k x n.  Returns new copies (W, Wt, H).

    H phase:  R = B^T W~, S = W^T W (see GRAM_*), then rows of H in turn.
    W phase:  T = B H^T, V = H H^T, then for each column j (d = V_jj + alpha_w):
              W~(:,j) <- V_jj/d W~(:,j) + (T(:,j) - W~ V(:,j)) / d   (no clip)
              W(:,j)  <- [Q W~(:,j) - beta_w / d]_+                 (lift, clip)
              W~(:,j) <- Q^T W(:,j)                                 (map back)
    The regularization terms follow Sec. 3.4 (readings R18, R19); with the
    default zero weights they vanish exactly.
    """
    Q = np.asarray(Q, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    W = np.array(W, dtype=np.float64)
    Wt = np.array(Wt, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    k = H.shape[0]

    def h_phase():
        R = B.T @ Wt
        if gram_mode == GRAM_FULL:
            S_num = S_scale = W.T @ W
        elif gram_mode == GRAM_LOWDIM:
            S_num = S_scale = Wt.T @ Wt
        elif gram_mode == GRAM_MIXED:
            S_num = Wt.T @ Wt
            S_scale = W.T @ W
        else:
            raise ValueError("unknown gram_mode")
        _h_rows(H, R, S_num, S_scale, reg.alpha_h, reg.beta_h)

    def w_phase():
        T = B @ H.T
        V = H @ H.T
        for j in range(k):
            v = V[j, j]
            d = v + reg.alpha_w
            if d > 0.0:
                Wt[:, j] = v / d * Wt[:, j] + (T[:, j] - Wt @ V[:, j]) / d
                W[:, j] = clip(Q @ Wt[:, j] - reg.beta_w / d)
                Wt[:, j] = Q.T @ W[:, j]

    if order == ORDER_H_FIRST:
        h_phase()
        w_phase()
    elif order == ORDER_W_FIRST:
        w_phase()
        h_phase()
    else:
        raise ValueError("unknown order")
    return W, Wt, H


def hals_sweep(X, W, H, order=ORDER_H_FIRST, reg=NO_REG):
    """One sweep of deterministic HALS with the residual-free rules of Sec. 3.1
    and their regularized form of Sec. 3.4 (reading R18):
    H(j,:) <- [s/(s+a_h) H(j,:) + ((X^T W)(:,j) - b_h - H^T (W^T W)(:,j)) / (s+a_h)]_+
    with s = (W^T W)_jj, and
    W(:,j) <- [v/(v+a_w) W(:,j) + ((X H^T)(:,j) - b_w - W (H H^T)(:,j)) / (v+a_w)]_+
    with v = (H H^T)_jj.  Returns new copies (W, H)."""
    X = np.asarray(X, dtype=np.float64)
    W = np.array(W, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    k = H.shape[0]

    def h_phase():
        S = W.T @ W
        _h_rows(H, X.T @ W, S, S, reg.alpha_h, reg.beta_h)

    def w_phase():
        V = H @ H.T
        P = X @ H.T
        for j in range(k):
            v = V[j, j]
            d = v + reg.alpha_w
            if d > 0.0:
                W[:, j] = clip(v / d * W[:, j] + (P[:, j] - reg.beta_w - W @ V[:, j]) / d)

    if order == ORDER_H_FIRST:
        h_phase()
        w_phase()
    elif order == ORDER_W_FIRST:
        w_phase()
        h_phase()
    else:
        raise ValueError("unknown order")
    return W, H


# ----------------------------------------------------------------------------
# Update orders (Sec. 3.2: the two cyclic orders and the shuffled order)
# ----------------------------------------------------------------------------
# An order is a sequence of block updates: entry e < k updates column e of W
# (with its lift and map-back in rHALS), entry e >= k updates row e - k of H.
# Reading R24: every block update takes the Gram and cross products of the
# factors as they are at that moment (in the blocked orders this equals
# forming them once per phase, as the other factor does not move within a
# phase); the shuffled order updates the components (W(:,j), H(j,:)) of the
# interleaved order in a random order per sweep, the permutation being an
# input.

def order_blocked(k, w_first=False):
    """W(:,1..k) then H(1..k,:) (w_first), or H rows then W columns
    (Algorithm 1's order)."""
    w = list(range(k))
    h = [k + j for j in range(k)]
    return w + h if w_first else h + w


def order_interleaved(k, perm=None):
    """W(:,j) -> H(j,:) for j = perm[0], perm[1], ... (the first cyclic order
    of Sec. 3.2 for perm = 0..k-1; the shuffled order for a random perm)."""
    perm = range(k) if perm is None else perm
    out = []
    for j in perm:
        out += [int(j), k + int(j)]
    return out


def rhals_sweep_ordered(Q, B, W, Wt, H, order):
    """One sweep of randomized HALS (Sec. 3.2, plain rules) with the block
    updates in the given order (reading R24).  For column j of W, with
    T(:,j) = B H(j,:)^T, V(:,j) = H H(j,:)^T and d = V_jj:
        W~(:,j) <- W~(:,j) + (T(:,j) - W~ V(:,j)) / d,
        W(:,j) <- [Q W~(:,j)]_+,  W~(:,j) <- Q^T W(:,j);
    for row j of H, with S(:,j) = W^T W(:,j), R(:,j) = B^T W~(:,j), s = S_jj:
        H(j,:) <- [H(j,:) + (R(:,j) - H^T S(:,j)) / s]_+.
    Blocks with a zero scale are skipped (reading R9).  Returns new copies
    (W, Wt, H)."""
    Q = np.asarray(Q, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    W = np.array(W, dtype=np.float64)
    Wt = np.array(Wt, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    k = H.shape[0]
    for e in order:
        if e < k:
            j = e
            T_j = B @ H[j, :]
            V_j = H @ H[j, :]
            d = V_j[j]
            if d > 0.0:
                Wt[:, j] = Wt[:, j] + (T_j - Wt @ V_j) / d
                W[:, j] = clip(Q @ Wt[:, j])
                Wt[:, j] = Q.T @ W[:, j]
        else:
            j = e - k
            S_j = W.T @ W[:, j]
            R_j = B.T @ Wt[:, j]
            d = S_j[j]
            if d > 0.0:
                H[j, :] = clip(H[j, :] + (R_j - H.T @ S_j) / d)
    return W, Wt, H


def hals_sweep_ordered(X, W, H, order):
    """One sweep of deterministic HALS (Sec. 3.1, plain rules) with the block
    updates in the given order: W(:,j) <- [W(:,j) + ((X H^T)(:,j) -
    W (H H^T)(:,j)) / (H H^T)_jj]_+ and H(j,:) <- [H(j,:) + ((X^T W)(:,j) -
    H^T (W^T W)(:,j)) / (W^T W)_jj]_+, the products taken from the current
    factors.  Returns new copies (W, H)."""
    X = np.asarray(X, dtype=np.float64)
    W = np.array(W, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    k = H.shape[0]
    for e in order:
        if e < k:
            j = e
            V_j = H @ H[j, :]
            d = V_j[j]
            if d > 0.0:
                W[:, j] = clip(W[:, j] + (X @ H[j, :] - W @ V_j) / d)
        else:
            j = e - k
            S_j = W.T @ W[:, j]
            d = S_j[j]
            if d > 0.0:
                H[j, :] = clip(H[j, :] + (X.T @ W[:, j] - H.T @ S_j) / d)
    return W, H


# ----------------------------------------------------------------------------
# Stopping measures and error (Sec. 3.3; tables of Sec. 4)
# ----------------------------------------------------------------------------

def _proj(G, F):
    """Projected gradient entries (Sec. 3.3): the gradient where the factor
    entry is positive, min(0, gradient) where it is zero."""
    return np.where(F > 0.0, G, np.minimum(G, 0.0))


def projected_gradient_sq(X, W, H, reg=NO_REG):
    """||grad^P f(W, H)||_F^2 for f = ||X - W H||_F^2 (Sec. 3.3), with the
    gradients W (H H^T) - X H^T and (W^T W) H - W^T X (factor 2 dropped,
    reading R10), plus alpha F + beta for the regularized cost (R18)."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    GW = W @ (H @ H.T) - X @ H.T + reg.alpha_w * W + reg.beta_w
    GH = (W.T @ W) @ H - W.T @ X + reg.alpha_h * H + reg.beta_h
    return float(np.sum(_proj(GW, W) ** 2) + np.sum(_proj(GH, H) ** 2))


def projected_gradient_sq_compressed(Q, B, W, Wt, H, reg=NO_REG):
    """Projected-gradient norm of Sec. 3.3 evaluated on the surrogate
    X^ = Q B without forming it (reading R10): the W gradient is
    W (H H^T) - Q (B H^T) and the H gradient is (W^T W) H - W~^T B, which
    equals (W^T W) H - W^T X^ when W~ = Q^T W; the regularized cost adds
    alpha F + beta to each (R18)."""
    Q = np.asarray(Q, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    Wt = np.asarray(Wt, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    GW = W @ (H @ H.T) - Q @ (B @ H.T) + reg.alpha_w * W + reg.beta_w
    GH = (W.T @ W) @ H - Wt.T @ B + reg.alpha_h * H + reg.beta_h
    return float(np.sum(_proj(GW, W) ** 2) + np.sum(_proj(GH, H) ** 2))


def objective(X, W, H, reg=NO_REG):
    """The regularized cost whose block minimisers are the rules of Sec. 3.4
    (reading R18): 1/2 ||X - W H||_F^2 + alpha/2 ||F||_F^2 + beta sum(F) for
    F = W, H (nonnegative factors, so sum(F) is the 1-norm)."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    E = X - W @ H
    return float(0.5 * np.sum(E * E)
                 + 0.5 * reg.alpha_w * np.sum(W * W) + reg.beta_w * np.sum(W)
                 + 0.5 * reg.alpha_h * np.sum(H * H) + reg.beta_h * np.sum(H))


def rel_error(X, W, H):
    """Relative reconstruction error ||X - W H||_F / ||X||_F (reading R11)."""
    X = np.asarray(X, dtype=np.float64)
    E = X - np.asarray(W, dtype=np.float64) @ np.asarray(H, dtype=np.float64)
    return float(np.linalg.norm(E) / np.linalg.norm(X))


# ----------------------------------------------------------------------------
# Drivers
# ----------------------------------------------------------------------------

def rhals(X, k, Omega, W0, H0, q=2, max_iter=100, tol=0.0,
          gram_mode=GRAM_FULL, order=ORDER_H_FIRST, trace=False, reg=NO_REG):
    """Randomized HALS, Algorithm 1.

    Omega (n x l), W0 (m x k) and H0 (k x n) are supplied by the caller; the
    width l is Omega's column count (already clamped, reading R1).  Runs sweeps
    until the projected-gradient ratio on X^ = Q B falls below tol (when
    tol > 0) or max_iter sweeps are done.  Returns (W, H, info) where info has
    Q, B, Wt, iters, rel_err (against X), pg_ratio and, when trace is set, the
    relative error after every sweep.
    """
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    if not (1 <= k < min(m, n)):
        raise ValueError("need 1 <= k < min(m, n)")
    Q, B = qb(X, Omega, q)
    W = np.array(W0, dtype=np.float64)
    H = np.array(H0, dtype=np.float64)
    Wt = Q.T @ W                                     # reading R4
    pg0 = projected_gradient_sq_compressed(Q, B, W, Wt, H, reg)
    it = 0
    ratio = 1.0
    errs = []
    while it < max_iter:
        W, Wt, H = rhals_sweep(Q, B, W, Wt, H, gram_mode, order, reg)
        it += 1
        if trace:
            errs.append(rel_error(X, W, H))
        if tol > 0.0:
            pg = projected_gradient_sq_compressed(Q, B, W, Wt, H, reg)
            ratio = pg / pg0 if pg0 > 0 else 0.0
            if ratio < tol:
                break
    if tol <= 0.0:
        pg = projected_gradient_sq_compressed(Q, B, W, Wt, H, reg)
        ratio = pg / pg0 if pg0 > 0 else 0.0
    info = dict(Q=Q, B=B, Wt=Wt, iters=it, rel_err=rel_error(X, W, H),
                pg_ratio=ratio, trace=errs)
    return W, H, info


def hals(X, W0, H0, max_iter=100, tol=0.0, order=ORDER_H_FIRST, trace=False, reg=NO_REG):
    """Deterministic HALS (Sec. 3.1) with the stopping rule of Sec. 3.3.
    Returns (W, H, info) with iters, rel_err, pg_ratio and an optional per-sweep
    error trace."""
    X = np.asarray(X, dtype=np.float64)
    W = np.array(W0, dtype=np.float64)
    H = np.array(H0, dtype=np.float64)
    pg0 = projected_gradient_sq(X, W, H, reg)
    it = 0
    ratio = 1.0
    errs = []
    while it < max_iter:
        W, H = hals_sweep(X, W, H, order, reg)
        it += 1
        if trace:
            errs.append(rel_error(X, W, H))
        if tol > 0.0:
            ratio = projected_gradient_sq(X, W, H, reg) / pg0 if pg0 > 0 else 0.0
            if ratio < tol:
                break
    if tol <= 0.0:
        ratio = projected_gradient_sq(X, W, H, reg) / pg0 if pg0 > 0 else 0.0
    return W, H, dict(iters=it, rel_err=rel_error(X, W, H), pg_ratio=ratio,
                      trace=errs)
