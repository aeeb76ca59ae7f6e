"""Host check of the block-pair scheme that takes each unordered pair of an
all-to-all network once (the library's k_pairs_sym and the step's sum of
partial sums). The pair term of Section 2.3.1, Algorithm 1, is odd in the
voltage difference, so the term of (j, i) is minus that of (i, j). Here the
scheme's assignment (column block J takes row blocks J + k mod B,
1 <= k <= B/2, k = B/2 only for J < B/2 when B is even; each block's own
pairs ordered) is followed in float64 with numpy for every block count up
to 12 and ragged sizes, and the summed partials are compared with the plain
all-pairs sum."""
import numpy as np
import pytest


def term(vi, vj):
    d = vi - vj
    return d * (0.8 * np.exp(-d * d / 100.0) + 0.2)


def scheme(v):
    n = len(v)
    B = (n + 63) // 64
    K = B // 2
    pad = np.full(B * 64, np.nan)
    pad[:n] = v
    rows = np.zeros(B * 64)
    taken = np.zeros((B, B), int)
    for J in range(B):
        KJ = (B - 1) // 2 + (1 if (B % 2 == 0 and J < B // 2) else 0)
        assert KJ <= K
        cj = pad[J * 64:(J + 1) * 64]
        for k in range(1, KJ + 1):
            I = (J + k) % B
            ri = pad[I * 64:(I + 1) * 64]
            t = term(ri[:, None], cj[None, :])           # rows of I against columns of J
            t[np.isnan(t)] = 0.0                         # padded cells contribute nothing
            rows[I * 64:(I + 1) * 64] += t.sum(axis=1)
            rows[J * 64:(J + 1) * 64] -= t.sum(axis=0)   # the mirrored terms
            taken[min(I, J), max(I, J)] += 1
        t = term(cj[:, None], cj[None, :])
        t[np.isnan(t)] = 0.0
        rows[J * 64:(J + 1) * 64] += t.sum(axis=1)
    return rows[:n], taken, B


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 128, 129, 200, 256, 320, 383, 384, 449, 512, 640, 700, 768])
def test_each_block_pair_once_and_sums_match(n):
    rs = np.random.default_rng(n)
    v = -60.0 + rs.uniform(-15.0, 15.0, n)
    got, taken, B = scheme(v)
    iu = np.triu_indices(B, 1)
    assert np.all(taken[iu] == 1), taken          # every pair of distinct blocks exactly once
    assert np.all(np.tril(taken) == 0)
    ref = term(v[:, None], v[None, :]).sum(axis=1)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9 * np.abs(term(v[:, None], v[None, :])).sum(axis=1).max())


def test_term_is_odd_bitwise_in_fp32():
    """The fp32 difference, square and factor of (j, i) equal those of (i, j)
    up to the sign of the difference, so the terms cancel exactly."""
    rs = np.random.default_rng(5)
    a = rs.uniform(-80, 20, 100000).astype(np.float32)
    b = rs.uniform(-80, 20, 100000).astype(np.float32)
    d1, d2 = a - b, b - a
    assert np.array_equal(d1, -d2)
    f1 = d1 * (np.float32(0.8) * np.exp2(-(d1 * d1) * np.float32(0.014426950408889634)) + np.float32(0.2))
    f2 = d2 * (np.float32(0.8) * np.exp2(-(d2 * d2) * np.float32(0.014426950408889634)) + np.float32(0.2))
    assert np.array_equal(f1, -f2)
