"""Seeded synthetic inputs for randomized-HALS tests and benchmarks.

This module holds input recipes only: random numbers, shapes and the
nonnegative low-rank-plus-noise matrices that stand in for the paper's
workloads.  It contains none of the factorisation's arithmetic, and both the
HIP library's tests and the FP64 oracle's tests take their inputs from here.

Streams: every workload has a master seed; each random array is drawn from a
NumPy PCG64 stream keyed by (seed, stream id[, chunk]) so that any row chunk of
a large matrix can be regenerated on its own:

    0 W* (per row chunk)   1 H*          2 noise (per row chunk)
    3 Omega                4 W0          5 H0
    6 sparsity mask of H*  7 batch shapes          8 row-chunk subsample

The batched workload (many independent NMFs of uneven shapes) draws its shapes
from stream 7 of its own seed; problem i is then an ordinary low-rank product
with seed ``batch_seed(seed, i)``.
"""

import numpy as np

S_WSTAR, S_HSTAR, S_NOISE, S_OMEGA, S_W0, S_H0, S_MASK, S_BATCH, S_SUB = 0, 1, 2, 3, 4, 5, 6, 7, 8

CHUNK_ROWS = 1000

# Workloads shaped like the paper's experiments (Sec. 4).  Sizes only; the
# data are synthetic nonnegative low-rank products plus clipped Gaussian noise.
WORKLOADS = {
    # small dense problem for FP64 parity: 500 x 400, rank-10 uniform factors,
    # absolute noise 0.01
    "small_500x400": dict(m=500, n=400, rank=10, k=10, p=20, q=2, sweeps=100,
                          noise_abs=0.01, noise_rel=0.0, density=1.0,
                          seed=101, dtype="f64"),
    # image-stack shape of the face-database experiment (Sec. 4.1):
    # 32,256 x 2,410, rank-40 product with 30%-dense H*, 1% relative noise
    "stack_32256x2410": dict(m=32256, n=2410, rank=40, k=16, p=20, q=2,
                             sweeps=500, noise_abs=0.0, noise_rel=0.01,
                             density=0.3, seed=102, dtype="f32"),
    # tall synthetic matrix of the performance study (Sec. 4.4):
    # 100,000 x 5,000, rank-50 uniform product, absolute noise 0.05
    "tall_100000x5000": dict(m=100000, n=5000, rank=50, k=50, p=20, q=2,
                             sweeps=200, noise_abs=0.05, noise_rel=0.0,
                             density=1.0, seed=103, dtype="f32"),
    # square synthetic matrix of the performance study (Sec. 4.4):
    # 25,000 x 25,000, rank-50 uniform product, absolute noise 0.05
    "square_25000x25000": dict(m=25000, n=25000, rank=50, k=50, p=20, q=2,
                               sweeps=200, noise_abs=0.05, noise_rel=0.0,
                               density=1.0, seed=106, dtype="f32"),
    # differentiation workload: 8,192 x 2,048, rank-32 uniform product, 1%
    # relative noise; T = 20 unrolled sweeps ("sweeps"), checkpoints every 5
    "diff_8192x2048": dict(m=8192, n=2048, rank=32, k=32, p=16, q=2, sweeps=20,
                           noise_abs=0.0, noise_rel=0.01, density=1.0,
                           seed=105, dtype="f32", ckpt_every=5),
}


def stream(seed, *key):
    """An independent NumPy generator for (seed, key...)."""
    ss = np.random.SeedSequence(int(seed), spawn_key=tuple(int(x) for x in key))
    return np.random.Generator(np.random.PCG64(ss))


def _factor_h(seed, r, n, density):
    H = stream(seed, S_HSTAR).random((r, n))
    if density < 1.0:
        H *= stream(seed, S_MASK).random((r, n)) < density
    return H


def _chunk_clean(seed, c, rows, Hs):
    Ws = stream(seed, S_WSTAR, c).random((rows, Hs.shape[0]))
    return Ws @ Hs


def _chunks(m):
    return [(c, c * CHUNK_ROWS, min(m, (c + 1) * CHUNK_ROWS))
            for c in range((m + CHUNK_ROWS - 1) // CHUNK_ROWS)]


def _noise_sigma(m, n, r, seed, noise_abs, noise_rel, density, Hs):
    if noise_rel <= 0.0:
        return float(noise_abs)
    ss = 0.0
    for c, r0, r1 in _chunks(m):
        ss += float(np.sum(_chunk_clean(seed, c, r1 - r0, Hs) ** 2))
    return float(noise_rel) * np.sqrt(ss / (m * n))


def low_rank_rows(m, n, rank, seed, noise_abs=0.0, noise_rel=0.0, density=1.0,
                  chunks=None, dtype=np.float64, threads=1):
    """Rows of X = max(0, W* H* + sigma N), W*, H* ~ U[0,1) (H* optionally
    masked to the given density), N standard normal.  sigma is noise_abs, or
    noise_rel times the RMS of the clean product.  With ``chunks`` (a list of
    row-chunk indices) only those chunks are generated and stacked."""
    Hs = _factor_h(seed, rank, n, density)
    sigma = _noise_sigma(m, n, rank, seed, noise_abs, noise_rel, density, Hs)
    all_chunks = _chunks(m)
    if chunks is None:
        sel = all_chunks
    else:
        sel = [all_chunks[int(c)] for c in chunks]
    rows = sum(r1 - r0 for _, r0, r1 in sel)
    X = np.empty((rows, n), dtype=dtype)
    offs = np.cumsum([0] + [r1 - r0 for _, r0, r1 in sel])

    def fill(i):
        c, r0, r1 = sel[i]
        blk = _chunk_clean(seed, c, r1 - r0, Hs)
        if sigma > 0.0:
            blk += sigma * stream(seed, S_NOISE, c).standard_normal(blk.shape)
        np.maximum(blk, 0.0, out=blk)
        X[offs[i]:offs[i + 1]] = blk

    if len(sel) > 4 and threads > 1:
        # chunks are independent streams, so threading does not change X
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(fill, range(len(sel))))
    else:
        for i in range(len(sel)):
            fill(i)
    return X


# Batched workload: independent problems with m ~ U[256, 4096], n ~ U[128, 2048],
# k ~ U{4..32}; each X is a rank-k uniform product plus 1% relative noise,
# clipped; p = 10, q = 2, 100 sweeps.
BATCH = dict(count=512, m=(256, 4096), n=(128, 2048), k=(4, 32), p=10, q=2, sweeps=100,
             noise_rel=0.01, seed=104)


def batch_seed(seed, i):
    return int(seed) * 1_000_003 + int(i)


def batch_shapes(count=None, seed=None, m=None, n=None, k=None):
    """(m, n, k) of each problem of the batched workload, drawn from stream 7."""
    b = BATCH
    count = b["count"] if count is None else count
    seed = b["seed"] if seed is None else seed
    m, n, k = m or b["m"], n or b["n"], k or b["k"]
    g = stream(seed, S_BATCH)
    ms = g.integers(m[0], m[1] + 1, count)
    ns = g.integers(n[0], n[1] + 1, count)
    ks = g.integers(k[0], k[1] + 1, count)
    return [(int(a), int(c), int(d)) for a, c, d in zip(ms, ns, ks)]


def batch_problem(i, m, n, k, p=None, seed=None, dtype=np.float32):
    """Problem i of a batch: (X, Omega, W0, H0) with l = min(k + p, m, n)."""
    b = BATCH
    p = b["p"] if p is None else p
    s = batch_seed(b["seed"] if seed is None else seed, i)
    X = low_rank_rows(m, n, k, s, noise_rel=b["noise_rel"])
    l = sketch_cols(k, p, m, n)
    Om = omega(n, l, s)
    W0, H0 = init_factors(m, n, k, s)
    return X.astype(dtype), Om.astype(dtype), W0.astype(dtype), H0.astype(dtype)


def workload(name):
    return dict(WORKLOADS[name])


def sketch_cols(k, p, m, n):
    return int(min(k + p, min(m, n)))


def omega(n, l, seed, dist="gaussian", dtype=np.float64):
    """Test matrix Omega (n x l): standard normal (default) or uniform [0, 1)."""
    g = stream(seed, S_OMEGA)
    if dist == "gaussian":
        A = g.standard_normal((n, l))
    elif dist == "uniform":
        A = g.random((n, l))
    else:
        raise ValueError(dist)
    return A.astype(dtype)


def init_factors(m, n, k, seed, dtype=np.float64):
    """Initial W0 (m x k) and H0 (k x n), i.i.d. uniform [0, 1)."""
    W0 = stream(seed, S_W0).random((m, k)).astype(dtype)
    H0 = stream(seed, S_H0).random((k, n)).astype(dtype)
    return W0, H0


def subsample_chunks(m, count, seed):
    """Sorted indices of ``count`` distinct row chunks, for a row subsample."""
    nchunks = (m + CHUNK_ROWS - 1) // CHUNK_ROWS
    idx = stream(seed, S_SUB).choice(nchunks, size=min(count, nchunks), replace=False)
    return np.sort(idx)


def make(name, rows_chunks=None, dtype=None, threads=1):
    """(X, Omega, W0, H0, params) for a named workload.  X, Omega, W0 and H0
    are produced in float64 and rounded once to the workload's storage type."""
    w = workload(name)
    dt = np.float64 if (dtype or w["dtype"]) == "f64" else np.float32
    X = low_rank_rows(w["m"], w["n"], w["rank"], w["seed"], w["noise_abs"],
                      w["noise_rel"], w["density"], chunks=rows_chunks,
                      dtype=dt, threads=threads)
    m = X.shape[0]
    n = w["n"]
    l = sketch_cols(w["k"], w["p"], m, n)
    Om = omega(n, l, w["seed"]).astype(dt)
    W0, H0 = init_factors(m, n, w["k"], w["seed"])
    return X, Om, W0.astype(dt), H0.astype(dt), w


def random_problem(m, n, rank, k, p, seed, noise_abs=0.01, dtype=np.float64,
                   density=1.0):
    """A small ad-hoc problem for tests: X, Omega, W0, H0 with l = k + p."""
    X = low_rank_rows(m, n, rank, seed, noise_abs=noise_abs, density=density)
    l = sketch_cols(k, p, m, n)
    Om = omega(n, l, seed)
    W0, H0 = init_factors(m, n, k, seed)
    return (X.astype(dtype), Om.astype(dtype), W0.astype(dtype), H0.astype(dtype))
