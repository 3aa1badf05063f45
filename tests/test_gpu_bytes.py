"""Bit-exact checks of the integer and byte work in the library, against
references written here from the published definitions (no code shared with
the library):

  - the FP32 -> BF16 cast (rnmf_cast_bf16) is round to nearest, ties to even,
    on the 16 discarded bits, for every class of input (ties, subnormals,
    overflow to infinity, zeros, NaN kept a NaN), with ragged widths and a
    leading dimension beyond the width;
  - the Philox4x32-10 block function (rnmf_philox4x32_10) reproduces the
    known-answer vectors published with the generator (Salmon et al., SC 2011)
    and a NumPy implementation of its rounds on random counters and keys;
  - the seeded matrices (rnmf_random): the uniform stream is exactly
    u(c0, c1) = ((c1 << 21) xor (c0 >> 11)) / 2^53 of the block output, the
    Gaussian stream is the Box-Muller transform of it within a few ulps
    (libm), and the uniform test matrix has the moments and the
    distribution of U[0, 1) (Kolmogorov-Smirnov);
  - Algorithm 1 with a generated uniform test matrix (Omega = NULL,
    omega_dist uniform; the Remark on the random test matrix) matches the
    oracle run on the same matrix.
"""

import numpy as np
import pytest

import oracle as o
import synth as s

torch = pytest.importorskip("torch")
rn = pytest.importorskip("paper_1711_02037_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not rn.available():
        raise RuntimeError("librnmf.so is not built")


# ---- BF16 round to nearest even, from the bit definition -------------------

def bf16_rne_bits(x):
    """uint16 BF16 patterns of float32 x: keep the top 16 bits and round on the
    16 discarded bits, to nearest with ties to the even kept pattern; a NaN is
    returned as 0x7FC0 (only its NaN-ness is compared)."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep = b >> 16
    rest = b & 0xFFFF
    up = (rest > 0x8000) | ((rest == 0x8000) & ((keep & 1) == 1))
    out = (keep + up.astype(np.uint64)) & 0xFFFF
    nan = np.isnan(x)
    out[nan] = 0x7FC0
    return out.astype(np.uint16)


def special_floats():
    bits = [0x00000000, 0x80000000,                  # zeros
            0x00000001, 0x00007FFF, 0x00008000, 0x00008001, 0x00018000, 0x007FFFFF,  # subnormals, ties
            0x00800000, 0x3F800000, 0x3F808000, 0x3F818000, 0x3F807FFF, 0x3F808001,  # 1 and ties around it
            0x7F7F7FFF, 0x7F7F8000, 0x7F7FFFFF,      # largest finite: down, tie to even (up), up to inf
            0x7F800000, 0xFF800000,                  # infinities
            0x7FC00000, 0x7F800001, 0xFFC00001,      # NaNs
            0xBF808000, 0xC0490FDB, 0x40490FDB]      # negative tie, -pi, pi
    return np.array(bits, dtype=np.uint32).view(np.float32)


# ragged rows, strided rows, and whole 8-element groups (packed, strided and
# a tall-wide case)
@pytest.mark.parametrize("m,n,ld", [(1, 25, 25), (7, 1003, 1003), (64, 1031, 1040), (129, 4096, 4099),
                                    (100, 1024, 1024), (33, 512, 520), (2100, 8192, 8192)])
def test_bf16_cast_is_round_to_nearest_even_bit_for_bit(m, n, ld):
    rng = np.random.default_rng(m * 100003 + n)
    bits = rng.integers(0, 2**32, size=(m, ld), dtype=np.uint64).astype(np.uint32)
    # a quarter of the entries are ties or one off a tie in the discarded half
    sel = rng.random((m, ld)) < 0.25
    bits[sel] = (bits[sel] & 0xFFFF0000) | rng.choice([0x7FFF, 0x8000, 0x8001], size=int(sel.sum())).astype(np.uint32)
    X = bits.view(np.float32).copy()
    sp = special_floats()
    X.reshape(-1)[: min(sp.size, X.size)] = sp[: min(sp.size, X.size)]
    Xd = torch.from_numpy(X).to(DEV)[:, :n]
    assert Xd.stride(0) == ld
    got = rn.cast_bf16(Xd).cpu().view(torch.int16).numpy().view(np.uint16)
    want = bf16_rne_bits(X[:, :n])
    nan = np.isnan(X[:, :n])
    assert np.array_equal(got[~nan], want[~nan])
    # a NaN stays a NaN (exponent all ones, nonzero mantissa)
    g = got[nan].astype(np.uint32)
    assert np.all(((g & 0x7F80) == 0x7F80) & ((g & 0x7F) != 0))
    # the same as torch's host conversion (round to nearest even) on the finite entries
    tb = torch.from_numpy(np.ascontiguousarray(X[:, :n])).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got[~nan], tb[~nan])


# ---- Philox4x32-10 ------------------------------------------------------------

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85


def philox_np(ctr, key):
    """Philox4x32-10 on arrays (count x 4 counters, count x 2 keys), from the
    round definition: (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2),
    hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)), keys bumped by the Weyl constants between
    rounds."""
    c = [ctr[:, i].astype(np.uint64) for i in range(4)]
    k0, k1 = key[:, 0].astype(np.uint64), key[:, 1].astype(np.uint64)
    mask = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & mask, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & mask]
        k0 = (k0 + np.uint64(W0)) & mask
        k1 = (k1 + np.uint64(W1)) & mask
    return np.stack(c, axis=1).astype(np.uint32)


# published known-answer vectors of Philox4x32-10: (counter, key, output)
KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


def _dev_i32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(DEV)


def test_philox_known_answer_vectors():
    ctr = np.array([c for c, _, _ in KAT], dtype=np.uint32)
    key = np.array([k for _, k, _ in KAT], dtype=np.uint32)
    want = np.array([r for _, _, r in KAT], dtype=np.uint32)
    got = rn.philox4x32_10(_dev_i32(ctr), _dev_i32(key)).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    assert np.array_equal(philox_np(ctr, key), want)  # the host reference agrees with the vectors


def test_philox_matches_round_definition_on_random_inputs():
    rng = np.random.default_rng(7)
    cnt = 100003
    ctr = rng.integers(0, 2**32, size=(cnt, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(cnt, 2), dtype=np.uint64).astype(np.uint32)
    got = rn.philox4x32_10(_dev_i32(ctr), _dev_i32(key)).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, philox_np(ctr, key))
    empty = torch.empty((0, 4), dtype=torch.int32, device=DEV)
    assert rn.philox4x32_10(empty, torch.empty((0, 2), dtype=torch.int32, device=DEV)).shape == (0, 4)


TAG = 0x524E4D46


def stream_words(rows, cols, seed, sid):
    e = np.arange(rows * cols, dtype=np.uint64)
    ctr = np.stack([e & np.uint64(0xFFFFFFFF), e >> np.uint64(32), np.full_like(e, sid), np.full_like(e, TAG)],
                   axis=1).astype(np.uint32)
    key = np.tile(np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint64), (e.size, 1)).astype(np.uint32)
    return philox_np(ctr, key)


def u53(lo, hi):
    return (((hi.astype(np.uint64) << np.uint64(21)) ^ (lo.astype(np.uint64) >> np.uint64(11))).astype(np.float64)
            / 9007199254740992.0)


@pytest.mark.parametrize("seed", [0, 103, 0xDEADBEEF12345678])
def test_seeded_streams_follow_the_block_function(seed):
    rows, cols = 517, 70
    c = stream_words(rows, cols, seed, 3)
    uni = u53(c[:, 0], c[:, 1]).reshape(rows, cols)
    got = rn.random(rows, cols, seed, 3, "uniform", dtype=torch.float64).cpu().numpy()
    assert np.array_equal(got, uni)                               # bit for bit
    got32 = rn.random(rows, cols, seed, 3, "uniform").cpu().numpy()
    assert np.array_equal(got32, uni.astype(np.float32))          # rounded once
    u1 = u53(c[:, 0], c[:, 1]) + 2.0 ** -53
    gau = (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u53(c[:, 2], c[:, 3]))).reshape(rows, cols)
    gg = rn.random(rows, cols, seed, 3, "gaussian", dtype=torch.float64).cpu().numpy()
    assert np.max(np.abs(gg - gau)) <= 1e-13 * max(1.0, np.max(np.abs(gau)))
    gc = rn.random(rows, cols, seed, 3, "gauss_clipped", dtype=torch.float64).cpu().numpy()
    assert np.array_equal(gc, np.where(gg > 0, gg, 0.0))
    # another stream id gives another matrix
    assert not np.array_equal(rn.random(rows, cols, seed, 4, "uniform", dtype=torch.float64).cpu().numpy(), uni)


def test_uniform_test_matrix_distribution():
    from scipy import stats
    n, l = 5000, 70
    U = rn.random(n, l, 103, 3, "uniform", dtype=torch.float64).cpu().numpy().ravel()
    assert U.min() >= 0.0 and U.max() < 1.0
    N = U.size
    # moments of U[0, 1): mean 1/2, variance 1/12, within 5 standard errors
    assert abs(U.mean() - 0.5) <= 5 * np.sqrt(1 / 12 / N)
    assert abs(U.var() - 1 / 12) <= 5 * np.sqrt(1 / 180 / N)
    assert stats.kstest(U, "uniform").pvalue > 1e-3
    # neighbouring elements are uncorrelated
    assert abs(np.corrcoef(U[:-1], U[1:])[0, 1]) <= 5 / np.sqrt(N)
    G = rn.random(n, l, 103, 3, "gaussian", dtype=torch.float64).cpu().numpy().ravel()
    assert stats.kstest(G, "norm").pvalue > 1e-3


def test_factorize_with_generated_uniform_test_matrix_matches_oracle():
    # Algorithm 1 with Omega drawn on the device from the uniform stream; the
    # oracle takes the same matrix, regenerated by the library's generator
    X, _, W0, H0 = s.random_problem(400, 300, 8, 8, 12, seed=31)
    k, p, q, seed = 8, 12, 2, 4242
    l = s.sketch_cols(k, p, *X.shape)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    W, H, info = rn.factorize(d(X), k, p, q, max_iter=30, precision="fp64", seed=seed, omega_dist="uniform",
                              W0=d(W0), H0=d(H0))
    Om = rn.random(X.shape[1], l, seed, 3, "uniform", dtype=torch.float64).cpu().numpy()
    Wo, Ho, io = o.rhals(X, k, Om, W0, H0, q=q, max_iter=30)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(W.cpu().numpy(), Wo) <= 1e-8 and rel(H.cpu().numpy(), Ho) <= 1e-8
    assert abs(info["rel_err"] - io["rel_err"]) <= 1e-10
