"""The seeded input generators: graph structure and distributions."""
import numpy as np
import pytest

from paper_1612_01501_amd import inputs as I


def _check_csr(n, rp, col):
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0)
    assert np.all(col != rows) and col.min() >= 0 and col.max() < n
    same_row = np.diff(rows) == 0
    assert np.all(np.diff(col)[same_row] > 0)                  # sorted, no duplicates
    a = np.sort(rows.astype(np.int64) * n + col)
    b = np.sort(col.astype(np.int64) * n + rows)
    np.testing.assert_array_equal(a, b)                       # symmetric


@pytest.mark.parametrize("n,p", [(300, 0.1), (2000, 0.01), (20000, 0.002)])
def test_erdos_renyi_structure_and_degree(n, p):
    rp, col = I.erdos_renyi_csr(n, p, 11)
    _check_csr(n, rp, col)
    deg = np.diff(rp)
    mean, var = (n - 1) * p, (n - 1) * p * (1 - p)
    assert abs(deg.mean() - mean) < 5 * np.sqrt(var / n) + 1e-9
    assert 0.8 * var < deg.var() < 1.2 * var


def test_seeded_draws_repeat():
    a = I.config1(0.1, seed=3, n=500)
    b = I.config1(0.1, seed=3, n=500)
    np.testing.assert_array_equal(a.col, b.col)
    np.testing.assert_array_equal(a.jitter, b.jitter)
    np.testing.assert_array_equal(a.bias, b.bias)
    assert np.abs(a.jitter).max() <= 1.0


def test_batch_recipe_ranges():
    nets = I.config3(seed=1, n_instances=40, n_max=300)
    assert all(64 <= n.n <= 300 for n in nets)
    assert all(0.01 <= n.g <= 0.08 for n in nets)
    assert all(2.0 <= n.pulses[0].amplitude <= 10.0 for n in nets)
    assert {n.conn for n in nets} <= {"uniform", "csr"}


def test_mlp_init_and_batch_shapes():
    w = I.mlp_init_params(1)
    assert w.shape == (20752,) and w.dtype == np.float32
    assert np.abs(w[:2048]).max() <= 0.25 and np.all(w[2048:2176] == 0)
    x, t = I.mlp_batch(32, 2)
    assert x.shape == (32, 16) and t.shape == (32, 16)
