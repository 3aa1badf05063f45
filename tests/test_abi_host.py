"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/rnmf.h declares, sizes workspaces, validates arguments
before touching a device, and maps a missing device to RNMF_ERR_HIP."""

import ctypes
import os
import re

import pytest

import paper_1711_02037_amd as rn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rnmf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rnmf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = rn.lib()
    names = declared_functions()
    assert len(names) >= 12
    for nm in names:
        assert hasattr(L, nm), nm
    assert sorted(rn.EXPORTS) == names


def test_status_strings_and_defaults():
    for s in range(11):
        assert rn.status_string(s)
    assert rn.status_string(99) == "unknown status"
    o = rn.Opts()
    rn.lib().rnmf_default_opts(ctypes.byref(o))
    assert (o.p, o.q, o.max_iter, o.prec, o.gram_mode, o.order) == (20, 2, 200, 1, 0, 0)
    assert o.flags & rn.FLAG_CHECK_INPUT


def test_sketch_width_clamps():
    assert rn.sketch_width(50, 20, 100000, 5000) == 70
    assert rn.sketch_width(10, 20, 500, 25) == 25
    assert rn.sketch_width(10, 20, 18, 400) == 18


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16"])
def test_workspace_sizes_grow_with_the_problem(prec):
    o = rn.make_opts(16, 20, 2, precision=prec)
    small = rn.workspace_bytes(rn.OP_FACTORIZE, 2000, 500, o)
    big = rn.workspace_bytes(rn.OP_FACTORIZE, 32256, 2410, o)
    assert 0 < small < big
    for op in (rn.OP_SKETCH, rn.OP_COMPRESS, rn.OP_HALS_STEP, rn.OP_REL_ERROR):
        assert 0 < rn.workspace_bytes(op, 32256, 2410, o) <= big
    assert big % 1 == 0


def test_workspace_query_rejects_bad_arguments():
    with pytest.raises(rn.RnmfError):
        rn.workspace_bytes(rn.OP_FACTORIZE, 100, 50, rn.make_opts(50, 20, 2))      # k >= min(m, n)
    with pytest.raises(rn.RnmfError):
        rn.workspace_bytes(rn.OP_FACTORIZE, 100000, 5000, rn.make_opts(100, 50, 2))  # l > 128
    with pytest.raises(rn.RnmfError):
        rn.workspace_bytes(rn.OP_FACTORIZE, 1000, 500, rn.make_opts(80, 20, 2))    # k > 64
    with pytest.raises(rn.RnmfError):
        rn.workspace_bytes(9, 100, 50, rn.make_opts(5, 5, 2))


def _call_factorize(o, m=100, n=80, ldx=80, xt=rn.F32, ws=ctypes.c_void_p(256), wsb=1 << 40):
    L = rn.lib()
    rep = rn.Report()
    p = ctypes.c_void_p(4096)
    return L.rnmf_factorize(p, xt, m, n, ldx, ctypes.byref(o), None, None, None, p, p, ctypes.byref(rep),
                            ws, wsb, None)


def test_arguments_are_checked_before_any_device_work():
    L = rn.lib()
    o = rn.make_opts(10, 5, 1)
    assert _call_factorize(o, ldx=79) == rn.ERR_SHAPE
    assert _call_factorize(o, xt=rn.F64) == rn.ERR_DTYPE
    assert _call_factorize(rn.make_opts(10, 5, 1, precision="fp64"), xt=rn.F32) == rn.ERR_DTYPE
    assert _call_factorize(rn.make_opts(100, 5, 1)) == rn.ERR_ARG
    assert _call_factorize(o, m=0) == rn.ERR_SHAPE
    bad = rn.make_opts(10, 5, 1)
    bad.reserved = 1
    assert _call_factorize(bad) == rn.ERR_ARG
    bad = rn.make_opts(10, 5, 1)
    bad.flags = 0x80
    assert _call_factorize(bad) == rn.ERR_ARG
    assert b"flag" in L.rnmf_last_error()
    bad = rn.make_opts(10, 5, 1)
    bad.tol = float("nan")
    assert _call_factorize(bad) == rn.ERR_ARG
    assert L.rnmf_factorize(None, rn.F32, 100, 80, 80, ctypes.byref(o), None, None, None, None, None, None,
                            None, 0, None) == rn.ERR_ARG


def test_missing_device_is_a_hip_error_not_a_crash():
    # On a host without a GPU the library must fail cleanly.
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    o = rn.make_opts(10, 5, 1)
    assert _call_factorize(o) == rn.ERR_HIP
    L = rn.lib()
    p = ctypes.c_void_p(4096)
    assert L.rnmf_hals_step(p, p, 100, 80, 15, 10, p, p, p, 1, ctypes.byref(o), None, p, 1 << 30,
                            None) == rn.ERR_HIP
    assert L.rnmf_cast_bf16(p, 10, 10, 10, p, None) in (rn.ERR_HIP, rn.OK)


def test_hals_step_validation():
    L = rn.lib()
    o = rn.make_opts(10, 5, 1)
    p = ctypes.c_void_p(4096)
    assert L.rnmf_hals_step(p, p, 100, 80, 15, 65, p, p, p, 1, ctypes.byref(o), None, p, 1 << 30,
                            None) == rn.ERR_ARG
    assert L.rnmf_hals_step(p, p, 100, 80, 200, 10, p, p, p, 1, ctypes.byref(o), None, p, 1 << 30,
                            None) == rn.ERR_SHAPE
    assert L.rnmf_hals_step(p, p, 100, 80, 15, 10, p, p, p, -1, ctypes.byref(o), None, p, 1 << 30,
                            None) == rn.ERR_ARG
    assert L.rnmf_hals_step(None, p, 100, 80, 15, 10, p, p, p, 1, ctypes.byref(o), None, p, 1 << 30,
                            None) == rn.ERR_ARG


def test_deterministic_hals_validation():
    L = rn.lib()
    p = ctypes.c_void_p(4096)
    o = rn.make_opts(10, 0, 0)
    assert rn.workspace_bytes(rn.OP_HALS, 1000, 300, o) > 0
    with pytest.raises(rn.RnmfError):
        rn.workspace_bytes(rn.OP_HALS, 1000, 300, rn.make_opts(10, 0, 0, precision="bf16"))
    with pytest.raises(rn.RnmfError):
        rn.workspace_bytes(rn.OP_HALS, 1000, 300, rn.make_opts(65, 0, 0))
    call = lambda opts, xt=rn.F32, k_ok=True, sweeps=1, ldx=300: L.rnmf_hals(
        p, xt, 1000, 300, ldx, p, p, sweeps, ctypes.byref(opts), p, 1 << 30, None)
    bad = rn.make_opts(10, 0, 0, tol=1e-4)
    assert call(bad) == rn.ERR_ARG
    assert b"tol" in L.rnmf_last_error()
    assert call(rn.make_opts(10, 0, 0, precision="bf16")) == rn.ERR_ARG
    assert call(rn.make_opts(301, 0, 0)) == rn.ERR_ARG
    assert call(o, sweeps=-1) == rn.ERR_ARG
    assert call(o, ldx=299) == rn.ERR_SHAPE
    assert call(o, xt=rn.F64) == rn.ERR_DTYPE
    assert L.rnmf_hals(None, rn.F32, 1000, 300, 300, p, p, 1, ctypes.byref(o), p, 1 << 30, None) == rn.ERR_ARG


def test_opts_layout_matches_the_header():
    # rnmf_opts: 4 x int32, double tol, uint64 seed, 6 x int32, 4 x double
    assert ctypes.sizeof(rn.Opts) == 88
    assert ctypes.sizeof(rn.Report) == 72
    assert rn.Opts.alpha_w.offset == 56 and rn.Opts.beta_h.offset == 80
    o = rn.Opts()
    rn.lib().rnmf_default_opts(ctypes.byref(o))
    assert (o.alpha_w, o.alpha_h, o.beta_w, o.beta_h) == (0.0, 0.0, 0.0, 0.0)


@pytest.mark.parametrize("bad", [{"alpha_w": -1.0}, {"beta_h": float("nan")}, {"alpha_h": float("inf")},
                                 {"beta_w": -1e-30}])
def test_regularization_weights_are_validated(bad):
    L = rn.lib()
    p = ctypes.c_void_p(4096)
    o = rn.make_opts(10, 20, 2, reg=bad)
    with pytest.raises(rn.RnmfError):
        rn.workspace_bytes(rn.OP_FACTORIZE, 2000, 500, o)
    assert L.rnmf_hals_step(p, p, 2000, 500, 30, 10, p, p, p, 1, ctypes.byref(o), None, p, 1 << 30,
                            None) == rn.ERR_ARG
    assert b"regularization" in L.rnmf_last_error()
    assert L.rnmf_hals(p, rn.F32, 2000, 500, 500, p, p, 1, ctypes.byref(o), p, 1 << 30, None) == rn.ERR_ARG
    with pytest.raises(ValueError):
        rn.make_opts(10, reg={"gamma": 1.0})
    good = rn.make_opts(10, 20, 2, reg={"alpha_w": 0.5, "beta_h": 2.0})
    assert rn.workspace_bytes(rn.OP_FACTORIZE, 2000, 500, good) > 0


def test_svd_init_validation():
    L = rn.lib()
    p = ctypes.c_void_p(4096)
    o = rn.make_opts(10, 20, 2)
    assert rn.workspace_bytes(rn.OP_SVD_INIT, 5000, 700, o) > 0
    with pytest.raises(rn.RnmfError):
        rn.workspace_bytes(rn.OP_SVD_INIT, 5000, 700, rn.make_opts(40, 60, 2))   # l = 100 > 96
    call = lambda m=5000, n=700, l=30, k=10, W=p: L.rnmf_svd_init(p, p, m, n, l, k, W, p, ctypes.byref(o), p,
                                                                   1 << 30, None)
    assert call(l=97) == rn.ERR_SHAPE
    assert call(l=30, m=20) == rn.ERR_SHAPE
    assert call(k=31) == rn.ERR_ARG
    assert call(k=0) == rn.ERR_ARG
    assert call(W=None) == rn.ERR_ARG
    # factorize: the flag needs l <= 96 and no W0 / H0
    big = rn.make_opts(40, 60, 2)
    big.flags |= rn.FLAG_SVD_INIT
    with pytest.raises(rn.RnmfError):
        rn.workspace_bytes(rn.OP_FACTORIZE, 5000, 700, big)
    f = rn.make_opts(10, 20, 2)
    f.flags |= rn.FLAG_SVD_INIT
    assert rn.workspace_bytes(rn.OP_FACTORIZE, 5000, 700, f) >= rn.workspace_bytes(rn.OP_FACTORIZE, 5000, 700, o)
    rep = rn.Report()
    assert L.rnmf_factorize(p, rn.F32, 5000, 700, 700, ctypes.byref(f), None, p, None, p, p, ctypes.byref(rep),
                            p, 1 << 40, None) == rn.ERR_ARG
    assert b"W0" in L.rnmf_last_error()


def test_batch_problem_layout_and_validation():
    assert ctypes.sizeof(rn.Problem) == 112
    L = rn.lib()
    assert L.rnmf_batch_workspace_bytes(512) > 512 * 104
    assert L.rnmf_batch_workspace_bytes(0) == 0
    good = dict(X=4096, Omega=4096, W0=4096, H0=4096, W=4096, H=4096, Q=4096, B=4096, Z=4096,
                m=1000, n=500, ldx=500, k=10, l=20, prec=rn.PREC["fp32"])

    def plan(**kw):
        d = dict(good, **kw)
        arr = (rn.Problem * 2)()
        for key, v in good.items():
            setattr(arr[0], key, v)
        for key, v in d.items():
            setattr(arr[1], key, v)
        return L.rnmf_batch_plan(arr, 2, ctypes.c_void_p(256), 1 << 30, None)

    assert plan(l=65) == rn.ERR_SHAPE
    assert b"problem 1" in L.rnmf_last_error()
    assert plan(l=600, m=500, n=500) == rn.ERR_SHAPE
    assert plan(k=33, l=40) == rn.ERR_ARG
    assert plan(k=21) == rn.ERR_ARG
    assert plan(ldx=499) == rn.ERR_SHAPE
    assert plan(Z=0) == rn.ERR_ARG
    assert plan(prec=0) == rn.ERR_ARG        # FP64 is not a batched precision
    assert plan(prec=rn.PREC["bf16"], reserved=1) == rn.ERR_ARG
    assert L.rnmf_batch_run(4, 33, 10, ctypes.c_void_p(256), 1 << 30, None) == rn.ERR_ARG
    assert L.rnmf_batch_run(4, 2, -1, ctypes.c_void_p(256), 1 << 30, None) == rn.ERR_ARG
    assert L.rnmf_batch_run(4, 2, 10, ctypes.c_void_p(256), 16, None) == rn.ERR_WORKSPACE


def test_backward_validation():
    L = rn.lib()
    p = ctypes.c_void_p(4096)
    o = rn.make_opts(8, 8, 0, precision="fp64")
    n1 = rn.backward_workspace_bytes(3000, 500, 16, 8, 10, 10, "fp64")
    n2 = rn.backward_workspace_bytes(3000, 500, 16, 8, 10, 3, "fp64")
    n3 = rn.backward_workspace_bytes(3000, 500, 16, 8, 10, 3, "fp32")
    assert n1 > n2 > n3 > 0     # more states per segment; FP32 states are half the size
    assert rn.backward_workspace_bytes(3000, 500, 16, 8, 0, 1, "fp64") > 0
    qb = lambda T=10, c=3, l=16, k=8, m=3000, oo=o: L.rnmf_backward_workspace_bytes(m, 500, l, k, T, c,
                                                                                   ctypes.byref(oo))
    assert qb(T=-1) == 0 and qb(c=-1) == 0 and qb(k=0) == 0 and qb(k=65, l=100) == 0
    assert qb(l=7) == 0 and qb(l=129) == 0 and qb(m=10) == 0

    def call(T=10, c=3, gX=None, gW=p, oo=o, l=16, ws_bytes=1 << 40, st=None):
        return L.rnmf_backward(p, p, 3000, 500, l, 8, p, p, p, T, c, st, gW, p, p, p, p, gX, ctypes.byref(oo), p,
                               ws_bytes, None)
    assert call(T=-1) == rn.ERR_ARG
    assert call(c=-1) == rn.ERR_ARG
    assert call(c=0) == rn.ERR_ARG              # ckpt_every = 0 needs recorded states
    assert call(c=3, st=p) == rn.ERR_ARG        # recorded states go with ckpt_every = 0
    assert call(c=0, st=p) == rn.ERR_HIP        # consistent: the missing device is reported
    # recorded states: no checkpoint or segment buffers
    assert rn.backward_workspace_bytes(3000, 500, 16, 8, 10, 0, "fp64") < n2
    assert call(gW=None) == rn.ERR_ARG
    assert call(l=4) == rn.ERR_SHAPE
    for field, value in (("gram_mode", 1), ("order", 1), ("alpha_h", 0.5), ("beta_w", 0.1)):
        bad = rn.make_opts(8, 8, 0, precision="fp64")
        setattr(bad, field, value)
        assert call(oo=bad) == rn.ERR_ARG, field
        assert qb(oo=bad) == 0, field
    # arguments check out: the missing device is reported, not a crash
    assert call(gX=p) == rn.ERR_HIP


def test_unroll_validation():
    L = rn.lib()
    p = ctypes.c_void_p(4096)
    o = rn.make_opts(8, 8, 0)
    call = lambda T=5, l=16, W=p, oo=o: L.rnmf_unroll(p, p, 3000, 500, l, 8, W, p, p, T, None, ctypes.byref(oo), p,
                                                       1 << 40, None)
    assert call(T=-1) == rn.ERR_ARG
    assert call(W=None) == rn.ERR_ARG
    assert call(l=7) == rn.ERR_SHAPE
    assert call() == rn.ERR_HIP
    assert rn.state_elems(3000, 500, 16, 8) == 3000 * 8 + 16 * 8 + 8 * 500


def test_hals_ordered_validation():
    L = rn.lib()
    p = ctypes.c_void_p(4096)
    k = 4
    o = rn.make_opts(k, 6, 0)
    assert L.rnmf_hals_ordered_workspace_bytes(3000, 500, 10, k) > 0
    assert L.rnmf_hals_ordered_workspace_bytes(3000, 500, 3, k) == 0

    def call(order, nsw=1, oo=o, W=p):
        arr = (ctypes.c_int32 * max(1, len(order)))(*order)
        return L.rnmf_hals_ordered(p, p, 3000, 500, 10, k, W, p, p, nsw, arr, ctypes.byref(oo), p, 1 << 30, None)
    good = rn.order_interleaved(k)
    assert sorted(good) == list(range(2 * k)) and rn.order_blocked(3, True) == [0, 1, 2, 3, 4, 5]
    assert call(good) == rn.ERR_HIP                      # arguments check out; no device here
    assert call(good[:-1] + [good[0]]) == rn.ERR_ARG     # a block twice
    assert call(good[:-1] + [2 * k]) == rn.ERR_ARG       # out of range
    assert call(good, nsw=-1) == rn.ERR_ARG
    assert call(good, W=None) == rn.ERR_ARG
    for field, value in (("gram_mode", 1), ("alpha_h", 0.5)):
        bad = rn.make_opts(k, 6, 0)
        setattr(bad, field, value)
        assert call(good, oo=bad) == rn.ERR_ARG, field


def test_generator_entry_points_validate_arguments():
    L = rn.lib()
    p = ctypes.c_void_p(4096)
    assert L.rnmf_random(None, rn.F32, 4, 4, 1, 3, 0, None) == rn.ERR_ARG
    assert L.rnmf_random(p, rn.F32, -1, 4, 1, 3, 0, None) == rn.ERR_SHAPE
    assert L.rnmf_random(p, rn.BF16, 4, 4, 1, 3, 0, None) == rn.ERR_DTYPE
    assert L.rnmf_random(p, rn.F32, 4, 4, 1, 3, 3, None) == rn.ERR_ARG
    assert L.rnmf_random(p, rn.F32, 4, 4, 1, 3, -1, None) == rn.ERR_ARG
    assert L.rnmf_random(p, rn.F64, 0, 4, 1, 3, 1, None) == rn.OK      # empty: nothing to launch
    assert L.rnmf_philox4x32_10(None, None, None, -1, None) == rn.ERR_SHAPE
    assert L.rnmf_philox4x32_10(None, p, p, 3, None) == rn.ERR_ARG
    assert L.rnmf_philox4x32_10(None, None, None, 0, None) == rn.OK
