"""GPU parity of the reverse pass through unrolled compressed sweeps
(rnmf_backward and the RandHALS autograd Function; readings R21-R23: Q fixed,
derivative of max(0, x) taken as 0 at 0, replaced blocks carry no derivative
of their old value) against the oracle's reference gradients
(oracle.adjoint.grads, the torch float64 unrolling pinned by central
differences).

Bars.  FP64 states: every gradient within 1e-9 of the reference, relative to
its largest entry.  The device and the reference run the same sweeps in a
different order of rounding (the device recomputes the forward with its own
sweep kernel), so the states agree to about 1e-15 and the reverse pass, a
product of T sweeps' Jacobians, adds a growth of at most a few hundred on these
shapes; no clip decision lies within 1e-12 of zero (measured: 1e-13 or
less).  FP32 states: 1e-4 relative Frobenius for a few sweeps.  The FP32
forward moves every state by about 1e-6 relative per sweep (one sweep is held
to 1e-5), and the reverse pass, which reads those states, carries that over
at the same order (measured: 2e-6 after 6 sweeps); the bar leaves room for a
clip decision that flips near zero, which changes a handful of entries.  For
the 20 sweeps of the differentiation workload the per-sweep drift adds up,
T x 1e-5 = 2e-4, and the bar is 1e-3 (measured: 2e-4 to 4e-4).
"""

import numpy as np
import pytest

import oracle as o
import synth as s

torch = pytest.importorskip("torch")
rn = pytest.importorskip("paper_1711_02037_amd")
from oracle import adjoint as A  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not rn.available():
        raise RuntimeError("librnmf.so is not built")


def dev(a, dt=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(DEV)


def host(t):
    return t.detach().to("cpu").to(torch.float64).numpy()


def relmax(a, b, floor=0.0):
    """Largest difference relative to the largest reference entry, or to
    `floor` where that is larger: a derivative that is zero in exact
    arithmetic (a replaced block's old value, reading R22) comes out of the
    reference as the difference of two equal terms, a residue of rounding
    times the upstream gradient, while the device writes an exact zero."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), floor, 1e-300))


def relf(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(m, n, k, l, seed):
    X = s.low_rank_rows(m, n, k + 2, seed, noise_abs=0.02)
    Q = o.range_finder(X, s.omega(n, l, seed), 1)
    W0, H0 = s.init_factors(m, n, k, seed)
    rng = s.stream(seed, 91)
    gW = rng.standard_normal((m, k))
    gH = rng.standard_normal((k, n))
    return X, Q, W0, H0, gW, gH


def run_device(X, Q, W0, H0, gW, gH, T, ckpt, dt):
    Qd = dev(Q, dt)
    B = dev(Q.T @ X, dt)
    W0d, H0d = dev(W0, dt), dev(H0, dt)
    Wt0 = dev(Q.T @ W0, dt)
    gB, gW0, gH0, gX = rn.backward(Qd, B, W0d, Wt0, H0d, T, dev(gW), dev(gH), ckpt, want_gX=True)
    torch.cuda.synchronize()
    return host(gB), host(gW0), host(gH0), host(gX)


CASES64 = [(300, 200, 6, 12, 7, 3, 601),     # two 256-row blocks of W, ragged; 3 segments, last one short
           (1000, 513, 16, 30, 5, 5, 602),   # one segment; n one past a 256-column block
           (257, 700, 40, 64, 4, 1, 603),    # k above 32 (the 64-row H reverse), one sweep per segment
           (90, 60, 1, 1, 3, 2, 604),        # k = l = 1
           (51200, 300, 8, 128, 3, 2, 605)]  # 200 rows x 128 FP64 per workgroup: Q slab streamed, not in LDS


@pytest.mark.parametrize("m,n,k,l,T,ckpt,seed", CASES64)
def test_backward_fp64_matches_reference(m, n, k, l, T, ckpt, seed):
    print(f"case m={m} n={n} k={k} l={l} T={T} ckpt={ckpt} seed={seed}", flush=True)
    X, Q, W0, H0, gW, gH = problem(m, n, k, l, seed)
    rX, rW0, rH0, _, _, _ = A.grads(Q, X, W0, H0, T, gW, gH)
    gB, gW0, gH0, gX = run_device(X, Q, W0, H0, gW, gH, T, ckpt, np.float64)
    fl = max(np.max(np.abs(gW)), np.max(np.abs(gH)))
    errs = (relmax(gX, rX, fl), relmax(gW0, rW0, fl), relmax(gH0, rH0, fl), relmax(gB, Q.T @ rX, fl))
    print("fp64 errors gX gW0 gH0 gB", errs, flush=True)
    assert max(errs) <= 1e-9, errs


def test_backward_fp32_matches_reference():
    m, n, k, l, T, ckpt, seed = 600, 400, 8, 20, 6, 4, 611
    print(f"case fp32 m={m} n={n} k={k} l={l} T={T}", flush=True)
    X, Q, W0, H0, gW, gH = problem(m, n, k, l, seed)
    # both sides start from the same FP32-rounded inputs
    X32, Q32 = X.astype(np.float32).astype(np.float64), Q.astype(np.float32).astype(np.float64)
    W32, H32 = W0.astype(np.float32).astype(np.float64), H0.astype(np.float32).astype(np.float64)
    rX, rW0, rH0, _, _, _ = A.grads(Q32, X32, W32, H32, T, gW, gH)
    gB, gW0, gH0, gX = run_device(X32, Q32, W32, H32, gW, gH, T, ckpt, np.float32)
    errs = (relf(gX, rX), relf(gW0, rW0), relf(gH0, rH0))
    print("fp32 errors gX gW0 gH0 (bar 1e-4)", errs, flush=True)
    assert max(errs) <= 1e-4, errs


def test_checkpoint_spacing_does_not_change_the_gradients():
    m, n, k, l, T, seed = 400, 300, 8, 16, 9, 621
    X, Q, W0, H0, gW, gH = problem(m, n, k, l, seed)
    outs = [run_device(X, Q, W0, H0, gW, gH, T, c, np.float64) for c in (1, 4, 9, 50)]
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


def test_recorded_states_give_the_recomputed_gradients():
    """rnmf_unroll's record and the recomputation inside rnmf_backward run
    the same one-sweep launches on the same inputs: identical gradients."""
    m, n, k, l, T, seed = 500, 350, 9, 18, 6, 625
    X, Q, W0, H0, gW, gH = problem(m, n, k, l, seed)
    for dt in (np.float64, np.float32):
        Qd, B = dev(Q, dt), dev(Q.T @ X, dt)
        W0d, Wt0, H0d = dev(W0, dt), dev(Q.T @ W0, dt), dev(H0, dt)
        W, Wt, H = W0d.clone(), Wt0.clone(), H0d.clone()
        states = rn.unroll(Qd, B, W, Wt, H, T)
        st = rn.state_elems(m, n, l, k)
        last = states[(T - 1) * st:T * st]
        assert torch.equal(last[:m * k], W.flatten()) and torch.equal(last[m * k + l * k:], H.flatten())
        a = rn.backward(Qd, B, W0d, Wt0, H0d, T, dev(gW), dev(gH), states=states, want_gX=True)
        b = rn.backward(Qd, B, W0d, Wt0, H0d, T, dev(gW), dev(gH), ckpt_every=4, want_gX=True)
        torch.cuda.synchronize()
        for u, v in zip(a, b):
            assert torch.equal(u, v)


def test_zero_sweeps_pass_the_upstream_gradients_through():
    m, n, k, l, seed = 200, 150, 5, 10, 631
    X, Q, W0, H0, gW, gH = problem(m, n, k, l, seed)
    gB, gW0, gH0, gX = run_device(X, Q, W0, H0, gW, gH, 0, 1, np.float64)
    assert np.array_equal(gW0, gW) and np.array_equal(gH0, gH)
    assert not gB.any() and not gX.any()


def test_unrolled_forward_matches_multi_sweep_launch():
    """The one-sweep launches that the reverse pass recomputes reach the
    states of one launch of T sweeps up to the order of rounding (the
    persistent launch carries sums from one sweep into the next, so the two
    are not bit-identical)."""
    m, n, k, l, T, seed = 700, 500, 12, 24, 6, 641
    X, Q, W0, H0, _, _ = problem(m, n, k, l, seed)
    for dt, bar in ((np.float64, 1e-12), (np.float32, 1e-4)):
        Qd, B = dev(Q, dt), dev(Q.T @ X, dt)
        W0d, Wt0, H0d = dev(W0, dt), dev(Q.T @ W0, dt), dev(H0, dt)
        W1, Wt1, H1 = rn.unrolled_forward(Qd, B, W0d, Wt0, H0d, T)
        W2, Wt2, H2 = W0d.clone(), Wt0.clone(), H0d.clone()
        rn.hals_step(Qd, B, W2, Wt2, H2, nsweeps=T)
        torch.cuda.synchronize()
        errs = [relf(host(a), host(b)) for a, b in ((W1, W2), (Wt1, Wt2), (H1, H2))]
        print(dt.__name__, "one-sweep launches vs one T-sweep launch", errs, flush=True)
        assert max(errs) <= bar, errs


@pytest.mark.parametrize("ckpt", [None, 2])
def test_autograd_function_matches_reference_loss_gradients(ckpt):
    """Loss ||X - W H||^2 + sum(H) (reading R23) through RandHALS: the loss
    itself is ordinary torch, the sweeps and their reverse are librnmf's
    (recorded states, or checkpoints every 2 sweeps)."""
    m, n, k, l, T, seed = 500, 300, 10, 20, 5, 651
    X, Q, W0, H0, _, _ = problem(m, n, k, l, seed)
    rX, rW0, rH0, rL, _, _ = A.grads(Q, X, W0, H0, T)
    Fn = rn.rand_hals_fn()
    Xd = dev(X).requires_grad_(True)
    W0d = dev(W0).requires_grad_(True)
    H0d = dev(H0).requires_grad_(True)
    W, H = Fn.apply(Xd, dev(Q), W0d, H0d, T, ckpt)
    E = Xd - W @ H
    L = (E * E).sum() + H.sum()
    L.backward()
    errs = (abs(float(L.detach()) - rL) / abs(rL), relmax(host(Xd.grad), rX), relmax(host(W0d.grad), rW0),
            relmax(host(H0d.grad), rH0))
    print("autograd errors L gX gW0 gH0", errs, flush=True)
    assert max(errs) <= 1e-9, errs


def test_autograd_gradients_match_device_central_differences():
    """Directional derivatives of the device forward, by central differences
    in FP64, against the device reverse pass; directions whose +-h step
    flips a clip decision of the reference forward are skipped."""
    m, n, k, l, T, seed = 256, 128, 8, 16, 5, 661
    X, Q, W0, H0, _, _ = problem(m, n, k, l, seed)
    Fn = rn.rand_hals_fn()
    Qd = dev(Q)

    def loss(Xa, Wa, Ha):
        W, H = Fn.apply(Xa, Qd, Wa, Ha, T, 2)
        E = Xa - W @ H
        return (E * E).sum() + H.sum()

    Xd, W0d, H0d = (dev(a).requires_grad_(True) for a in (X, W0, H0))
    loss(Xd, W0d, H0d).backward()
    g = [host(t.grad) for t in (Xd, W0d, H0d)]
    rng = s.stream(seed, 92)
    base = A.active_sets(Q, X, W0, H0, T)
    h, checked = 1e-6, 0
    for trial in range(6):
        d = [rng.standard_normal(a.shape) for a in (X, W0, H0)]
        pts = [[a + sg * h * da for a, da in zip((X, W0, H0), d)] for sg in (1, -1)]
        if not all(all(np.array_equal(u, v) for u, v in zip(base, A.active_sets(Q, *pt, T))) for pt in pts):
            continue
        with torch.no_grad():
            lp, lm = (float(loss(*[dev(a) for a in pt])) for pt in pts)
        fd = (lp - lm) / (2 * h)
        an = float(sum(np.sum(gi * di) for gi, di in zip(g, d)))
        print(f"direction {trial}: fd {fd:.10e} analytic {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (trial, fd, an)
        checked += 1
    assert checked >= 3


def test_face_stack_size_fp64():
    """The face-database image-stack shape (32,256 x 2,410, k = 16, l = 36)
    with FP64 states, 6 sweeps in checkpoints of 4."""
    w = s.workload("stack_32256x2410")
    m, n, k = w["m"], w["n"], w["k"]
    l = k + w["p"]
    T, ckpt, seed = 6, 4, 671
    print(f"case face stack m={m} n={n} k={k} l={l} T={T}", flush=True)
    X = s.low_rank_rows(m, n, w["rank"], w["seed"], noise_rel=w["noise_rel"], density=w["density"])
    Q = o.range_finder(X, s.omega(n, l, w["seed"]), w["q"])
    W0, H0 = s.init_factors(m, n, k, seed)
    rng = s.stream(seed, 91)
    gW, gH = rng.standard_normal((m, k)), rng.standard_normal((k, n))
    rX, rW0, rH0, _, _, _ = A.grads(Q, X, W0, H0, T, gW, gH)
    gB, gW0, gH0, gX = run_device(X, Q, W0, H0, gW, gH, T, ckpt, np.float64)
    errs = (relmax(gX, rX), relmax(gW0, rW0), relmax(gH0, rH0))
    print("face stack fp64 errors gX gW0 gH0", errs, flush=True)
    assert max(errs) <= 1e-9, errs


def c5_inputs():
    """The differentiation workload: 8,192 x 2,048 FP32 X (rank-32 uniform
    product plus 1% relative noise), k = 32, l = 48, Q from the oracle's range
    finder with q = 2 on the FP32 X, FP32-rounded Q, W0, H0."""
    w = s.workload("diff_8192x2048")
    X, Om, W0, H0, _ = s.make("diff_8192x2048")
    X64 = X.astype(np.float64)
    Q = o.range_finder(X64, Om.astype(np.float64), w["q"]).astype(np.float32).astype(np.float64)
    return (w, X64, Q, W0.astype(np.float64), H0.astype(np.float64))


def device_loss_grads(X, Q, W0, H0, T, ckpt, dt):
    Fn = rn.rand_hals_fn()
    Xd, W0d, H0d = (dev(a, dt).requires_grad_(True) for a in (X, W0, H0))
    W, H = Fn.apply(Xd, dev(Q, dt), W0d, H0d, T, ckpt)
    E = Xd.double() - W.double() @ H.double()
    L = (E * E).sum() + H.double().sum()
    L.backward()
    torch.cuda.synchronize()
    return float(L.detach()), host(Xd.grad), host(W0d.grad), host(H0d.grad)


def device_masks(X, Q, W0, H0, T):
    """Activities (W_t > 0, H_t > 0) of the device's own FP32 trajectory: the
    states that the autograd forward records (same inputs, same calls)."""
    Qd = dev(Q, np.float32)
    B = rn.compress(dev(X, np.float32), Qd)
    W0d, H0d = dev(W0, np.float32), dev(H0, np.float32)
    Wt0 = rn.compress(W0d, Qd)
    m, l = Q.shape
    k, n = H0.shape
    st = rn.unroll(Qd, B, W0d.clone(), Wt0.clone(), H0d.clone(), T, record=True).cpu().numpy()
    per = rn.state_elems(m, n, l, k)
    masks = []
    for i in range(T):
        blk = st[i * per:(i + 1) * per]
        masks.append((blk[:m * k].reshape(m, k) > 0, blk[m * k + l * k:].reshape(k, n) > 0))
    return masks


def test_c5_fp32_checkpointed_autograd_matches_reference():
    """The differentiation workload as configured: FP32, T = 20, checkpoints
    every 5 sweeps, loss ||X - W H||^2 + sum(H).  The reference gradient is the
    float64 unrolling on the linear piece that the device's own FP32
    trajectory lies on (its activities, reading R22): FP32 rounding moves a
    few pre-clip values across zero, and each such flip changes the
    derivative by a finite amount, so the plain float64 reference (its own
    activities) is reported beside it but not held to the bar."""
    w, X, Q, W0, H0 = c5_inputs()
    T, ckpt = w["sweeps"], w["ckpt_every"]
    print(f"case C5 fp32 m={X.shape[0]} n={X.shape[1]} k={w['k']} l={Q.shape[1]} T={T} ckpt={ckpt}", flush=True)
    L, gX, gW0, gH0 = device_loss_grads(X, Q, W0, H0, T, ckpt, np.float32)
    masks = device_masks(X, Q, W0, H0, T)
    ref_masks = A.trajectory_masks(Q, X, W0, H0, T)
    flips = sum(int((a != b).sum()) + int((c != d).sum()) for (a, c), (b, d) in zip(masks, ref_masks))
    mX, mW0, mH0, mL = A.grads_masked(Q, X, W0, H0, T, masks)
    errs = (abs(L - mL) / abs(mL), relf(gX, mX), relf(gW0, mW0), relf(gH0, mH0))
    rX, rW0, rH0, rL, _, _ = A.grads(Q, X, W0, H0, T)
    plain = (abs(L - rL) / abs(rL), relf(gX, rX), relf(gW0, rW0), relf(gH0, rH0))
    print(f"C5 fp32 errors L gX gW0 gH0 on the device's piece {errs}; against the float64 trajectory {plain} "
          f"({flips} of {sum(a.size + c.size for a, c in masks)} activities differ)", flush=True)
    assert max(errs) <= 1e-3, errs


def test_c5_fp64_matches_reference_and_slice_central_differences():
    """The differentiation workload with FP64 states: gradients against the
    reference (1e-9), and directional derivatives along directions supported
    on a 256 x 128 slice of X (rows and columns 0..) and the matching rows of
    W0 and columns of H0, by central differences of the device forward."""
    w, X, Q, W0, H0 = c5_inputs()
    T, ckpt = w["sweeps"], w["ckpt_every"]
    rX, rW0, rH0, rL, _, _ = A.grads(Q, X, W0, H0, T)
    L, gX, gW0, gH0 = device_loss_grads(X, Q, W0, H0, T, ckpt, np.float64)
    errs = (abs(L - rL) / abs(rL), relmax(gX, rX), relmax(gW0, rW0), relmax(gH0, rH0))
    print("C5 fp64 errors L gX gW0 gH0", errs, flush=True)
    assert max(errs) <= 1e-9, errs
    Fn = rn.rand_hals_fn()
    Qd = dev(Q)

    def loss(Xa, Wa, Ha):
        with torch.no_grad():
            Xt, Wt_, Ht = dev(Xa), dev(Wa), dev(Ha)
            W, H = Fn.apply(Xt, Qd, Wt_, Ht, T, ckpt)
            E = Xt - W @ H
            return float((E * E).sum() + H.sum())

    rng = s.stream(w["seed"], 93)
    base = A.active_sets(Q, X, W0, H0, T)
    h, checked = 1e-6, 0
    for trial in range(4):
        dX = np.zeros_like(X); dX[:256, :128] = rng.standard_normal((256, 128))
        dW = np.zeros_like(W0); dW[:256] = rng.standard_normal((256, W0.shape[1]))
        dH = np.zeros_like(H0); dH[:, :128] = rng.standard_normal((H0.shape[0], 128))
        pts = [(X + sg * h * dX, W0 + sg * h * dW, H0 + sg * h * dH) for sg in (1, -1)]
        if not all(all(np.array_equal(u, v) for u, v in zip(base, A.active_sets(Q, *pt, T))) for pt in pts):
            print(f"direction {trial}: a clip decision flips within +-h, skipped", flush=True)
            continue
        fd = (loss(*pts[0]) - loss(*pts[1])) / (2 * h)
        an = float(np.sum(gX * dX) + np.sum(gW0 * dW) + np.sum(gH0 * dH))
        print(f"direction {trial}: fd {fd:.10e} analytic {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (trial, fd, an)
        checked += 1
    assert checked >= 2
