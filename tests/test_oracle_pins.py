"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not against the oracle itself.

Paper passages: Section 2.2 (synchronous step from the previous state,
dt = 50 us, one input per neuron per step, axon voltage as output),
Section 2.3.1 with Algorithm 1 (gap-junction current), Section 3 (validation:
a current pulse of about 500 steps makes every cell fire, identical initial
states keep cells in synchrony).
"""
import math
import os

import numpy as np
import pytest

from paper_1612_01501_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
VD, CA, R, S, Q, VS, KK, LL, HH, NN, XX, VA, HA, XA = range(14)
P = {name: k for k, name in enumerate(I.PARAM_NAMES)}


def _two_cells(dv, w=0.04):
    return I.Network(n=2, conn="dense", w_dense=np.array([[0.0, w], [w, 0.0]]))


# ----------------------------------------------------------------- gap term
def test_gap_pair_closed_form(o64):
    """f(dV) against hand-written values of 0.8*exp(-dV^2/100)+0.2."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "gap_pair_values.txt"))
            if l.strip() and not l.startswith("#")]
    w = 0.04
    for dv_s, f_s in rows:
        dv, f = float(dv_s), float(f_s)
        net = _two_cells(dv, w)
        ig = o64.gap(net, np.array([dv, 0.0]))
        assert ig[0] == pytest.approx(w * dv * f, rel=1e-14, abs=1e-300)


def test_gap_small_dv_is_linear(o64):
    """f(0) = 1: for |dV| <= 0.01 mV the term is w*dV to 1e-6 relative."""
    for dv in (1e-2, -3e-3, 1e-5):
        ig = o64.gap(_two_cells(dv), np.array([dv, 0.0]))
        assert abs(ig[0] / (0.04 * dv) - 1.0) <= 1e-6


def test_gap_large_dv_tends_to_linear_fifth(o64):
    """f -> 0.2 as |dV| -> inf."""
    ig = o64.gap(_two_cells(100.0), np.array([100.0, 0.0]))
    assert ig[0] == pytest.approx(0.04 * 100.0 * 0.2, rel=1e-12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gap_antisymmetry_bitwise(prec, o64, o32):
    o = o64 if prec == "f64" else o32
    rs = np.random.default_rng(1)
    for _ in range(50):
        v = rs.uniform(-80, 40, 2)
        ig = o.gap(_two_cells(0.0, 0.037), v)
        assert ig[0] == -ig[1]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gap_sum_rule_symmetric(prec, o64, o32):
    """Symmetric w: sum_i I_gap,i = 0 up to n*eps times the sum of |terms|."""
    o = o64 if prec == "f64" else o32
    eps = np.finfo(o.np_real).eps
    n = 40
    rs = np.random.default_rng(2)
    w = rs.uniform(0, 0.1, (n, n))
    w = np.triu(w, 1)
    w = w + w.T
    v = rs.uniform(-70, -40, n)
    net = I.Network(n=n, conn="dense", w_dense=w)
    ig = o.gap(net, v).astype(np.float64)
    dv = v[:, None] - v[None, :]
    mag = np.abs(w * dv).sum()
    assert abs(ig.sum()) <= 4 * n * eps * mag


def test_gap_brute_force_tiny(o64):
    """N <= 8 with pure-Python loops over a random dense w."""
    rs = np.random.default_rng(3)
    for n in (1, 3, 8):
        w = rs.uniform(0, 0.1, (n, n))
        v = rs.uniform(-70, -30, n)
        ig = o64.gap(I.Network(n=n, conn="dense", w_dense=w), v)
        for i in range(n):
            s = 0.0
            for j in range(n):
                d = v[i] - v[j]
                s += w[i, j] * d * (0.8 * math.exp(-d * d / 100.0) + 0.2)
            assert ig[i] == pytest.approx(s, rel=1e-13, abs=1e-15)


def test_gap_formats_agree(o64):
    """Uniform all-to-all == dense (w = g off-diagonal) == complete CSR."""
    n = 17
    v = np.random.default_rng(4).uniform(-70, -40, n)
    g = 0.03
    wd = np.full((n, n), g)
    np.fill_diagonal(wd, 0.0)
    rp, col = I.complete_csr(n)
    a = o64.gap(I.Network(n=n, conn="uniform", g=g), v)
    b = o64.gap(I.Network(n=n, conn="dense", w_dense=wd), v)
    c = o64.gap(I.Network(n=n, conn="csr", g=g, row_ptr=rp, col=col), v)
    d = o64.gap(I.Network(n=n, conn="csr", g=0.0, row_ptr=rp, col=col,
                          w_csr=np.full(len(col), g)), v)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(a, d)


def test_gap_reverse_order_close(o32):
    n = 64
    v = np.random.default_rng(5).uniform(-70, -40, n).astype(np.float32)
    net = I.Network(n=n, conn="uniform", g=0.04)
    a = o32.gap(net, v).astype(np.float64)
    b = o32.gap(net, v, reverse_j=True).astype(np.float64)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-5 * np.abs(a).max())


# ----------------------------------------------------------------- simplified gap junctions
# Section 2.3.2 (SGJ): a connection is a weighted accumulator of the voltage
# difference, I_gap,i = sum_j w_ij (Vd_i - Vd_j).

def test_sgj_is_laplacian_times_vd(o64):
    """Dense and CSR: I = (diag(W 1) - W) Vd, the weighted graph Laplacian
    applied to Vd, by a numpy matrix product."""
    rs = np.random.default_rng(11)
    for n in (1, 5, 33):
        w = rs.uniform(0, 0.1, (n, n)) * (rs.uniform(size=(n, n)) < 0.4)
        v = rs.uniform(-70, -30, n)
        lap = np.diag(w.sum(axis=1)) - w
        want = lap @ v
        got = o64.gap(I.Network(n=n, conn="dense", w_dense=w, gap="sgj"), v)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
        rows, cols = np.nonzero(w)
        rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int64)
        got = o64.gap(I.Network(n=n, conn="csr", row_ptr=rp, col=cols.astype(np.int32),
                                w_csr=w[rows, cols], gap="sgj"), v)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_sgj_uniform_closed_form(o64):
    """All-to-all with one conductance g: I_i = g (N Vd_i - sum_j Vd_j)."""
    n, g = 97, 0.04
    v = np.random.default_rng(12).uniform(-70, -40, n)
    got = o64.gap(I.Network(n=n, conn="uniform", g=g, gap="sgj"), v)
    np.testing.assert_allclose(got, g * (n * v - v.sum()), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sgj_sum_rule_symmetric(prec, o64, o32):
    """Symmetric w: the currents sum to zero up to rounding."""
    o = o64 if prec == "f64" else o32
    eps = np.finfo(o.np_real).eps
    n = 40
    rs = np.random.default_rng(13)
    w = np.triu(rs.uniform(0, 0.1, (n, n)), 1)
    w = w + w.T
    v = rs.uniform(-70, -40, n)
    ig = o.gap(I.Network(n=n, conn="dense", w_dense=w, gap="sgj"), v).astype(np.float64)
    assert abs(ig.sum()) <= 4 * n * eps * np.abs(w * (v[:, None] - v[None, :])).sum()


def test_sgj_is_small_dv_limit_of_rgj(o64):
    """The realistic factor 0.8 exp(-dV^2/100) + 0.2 is 1 at dV = 0 and
    1 - f <= 0.8 dV^2/100: for voltage spreads of 1e-3 mV each row of the two
    forms differs by at most that times the row's sum of |w dV|; at spreads
    of 100 mV the realistic one tends to a fifth of the simplified."""
    n = 20
    rs = np.random.default_rng(14)
    w = rs.uniform(0, 0.1, (n, n))
    v = -60.0 + rs.uniform(-1e-3, 1e-3, n)
    a = o64.gap(I.Network(n=n, conn="dense", w_dense=w), v)
    b = o64.gap(I.Network(n=n, conn="dense", w_dense=w, gap="sgj"), v)
    dv = v[:, None] - v[None, :]
    bound = 0.8 * (dv ** 2).max() / 100.0 * np.abs(w * dv).sum(axis=1) + 1e-15
    assert np.all(np.abs(a - b) <= bound)
    assert np.abs(a - b).max() > 0.0        # the two forms are not the same
    two = np.array([[0.0, 0.04], [0.04, 0.0]])
    vv = np.array([100.0, 0.0])
    ra = o64.gap(I.Network(n=2, conn="dense", w_dense=two), vv)
    rb = o64.gap(I.Network(n=2, conn="dense", w_dense=two, gap="sgj"), vv)
    assert ra[0] == pytest.approx(0.2 * rb[0], rel=1e-12)


def test_sgj_formats_agree(o64):
    """Uniform == dense (w = g off-diagonal) == complete CSR, bitwise."""
    n = 17
    v = np.random.default_rng(15).uniform(-70, -40, n)
    g = 0.03
    wd = np.full((n, n), g)
    np.fill_diagonal(wd, 0.0)
    rp, col = I.complete_csr(n)
    a = o64.gap(I.Network(n=n, conn="uniform", g=g, gap="sgj"), v)
    b = o64.gap(I.Network(n=n, conn="dense", w_dense=wd, gap="sgj"), v)
    c = o64.gap(I.Network(n=n, conn="csr", g=g, row_ptr=rp, col=col, gap="sgj"), v)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)


# ----------------------------------------------------------------- per-cell parameters
# Section 2.2: each neuron carries its own 20 conductances and reversal
# potentials.

def _het_params(n, seed):
    """Per-cell values: the defaults with gCaL, gH and gKCa scaled by U[0.7, 1.3]."""
    rs = np.random.default_rng(seed)
    cp = np.tile(I.DEFAULT_PARAMS, (n, 1))
    for name in ("g_CaL", "g_h", "g_KCa"):
        cp[:, P[name]] *= rs.uniform(0.7, 1.3, n)
    return cp


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cell_params_all_equal_is_the_network_run(prec, o64, o32):
    o = o64 if prec == "f64" else o32
    net = I.config1(0.1, seed=2, n=80)
    a = o.run(net, 300)
    net.cell_params = np.tile(net.params, (net.n, 1))
    b = o.run(net, 300)
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_array_equal(a["counts"], b["counts"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_uncoupled_heterogeneous_cells_are_their_own_networks(prec, o64, o32):
    """Cell i of an uncoupled network with per-cell values evolves exactly as
    a one-cell network with cell i's values (its own rest state, the pulse)."""
    o = o64 if prec == "f64" else o32
    n = 6
    cp = _het_params(n, 5)
    net = I.Network(n=n, conn="none", cell_params=cp, pulses=[I.Pulse(50, 250, 5.0)])
    x0 = o.initial_state(net)
    got = o.run(net, 400, x0=x0)["x"]
    for i in range(n):
        one = I.Network(n=1, conn="none", params=cp[i], pulses=[I.Pulse(50, 250, 5.0)])
        want = o.run(one, 400, x0=o.initial_state(one))["x"]
        np.testing.assert_array_equal(got[:, i], want[:, 0])
    assert np.unique(got[0]).size == n          # the cells differ


# ----------------------------------------------------------------- network invariants
@pytest.mark.parametrize("conn", ["uniform", "dense", "csr"])
def test_identical_cells_stay_in_sync(conn, o64, o32):
    """Section 3: identical initial states keep every cell identical (all dV = 0)."""
    n = 12
    kw = {}
    if conn == "dense":
        kw["w_dense"] = np.random.default_rng(6).uniform(0, 0.08, (n, n))
    if conn == "csr":
        kw["row_ptr"], kw["col"] = I.erdos_renyi_csr(n, 0.5, 7)
        kw["w_csr"] = np.random.default_rng(8).uniform(0, 0.08, len(kw["col"]))
    net = I.Network(n=n, conn=conn, g=0.05, pulses=[I.Pulse(100, 600, 6.0)], **kw)
    for o in (o64, o32):
        r = o.run(net, 1500)
        x = r["x"]
        for i in range(1, n):
            np.testing.assert_array_equal(x[:, i], x[:, 0])
        assert len(set(r["counts"].tolist())) == 1 and r["counts"][0] >= 1


def test_zero_coupling_gives_independent_cells(o64):
    n = 6
    jit = I.voltage_jitter(n, 11)
    base = dict(jitter=jit, pulses=[I.Pulse(100, 600, 6.0)], bias=np.linspace(-0.5, 0.5, n))
    a = o64.run(I.Network(n=n, conn="uniform", g=0.0, **base), 1200)
    b = o64.run(I.Network(n=n, conn="none", **base), 1200)
    np.testing.assert_array_equal(a["x"], b["x"])
    full = o64.initial_state(I.Network(n=n, conn="none", jitter=jit))
    for i in range(n):
        single = I.Network(n=1, conn="none", bias=base["bias"][i:i + 1],
                           pulses=[I.Pulse(100, 600, 6.0)])
        r = o64.run(single, 1200, x0=full[:, i:i + 1])
        np.testing.assert_array_equal(r["x"][:, 0], b["x"][:, i])


def test_gap_coupling_is_diffusive(o64):
    """dV = own - neighbour, subtracted in the dendrite: coupling pulls the two
    dendrites together (their difference after 1 ms shrinks with g)."""
    x0 = o64.initial_state(I.Network(n=2, conn="none"))
    x0[VD, 0] += 3.0
    d = []
    for g in (0.0, 0.04):
        r = o64.run(I.Network(n=2, conn="uniform", g=g), 20, x0=x0)
        d.append(abs(r["x"][VD, 0] - r["x"][VD, 1]))
    assert d[1] < d[0]


def test_symmetric_network_gap_sums_to_zero_along_run(o64):
    net = I.config1(0.2, seed=1, n=64)
    x = o64.run(net, 200)["x"]
    ig = o64.gap(net, x[VD])
    assert abs(ig.sum()) < 1e-12 * max(1.0, np.abs(ig).sum())


# ----------------------------------------------------------------- cell model
def test_single_cell_rest_no_spike_and_oscillates(o64):
    """Section 2.2: cells oscillate even when not spiking. Without input the
    cell stays subthreshold (no axon spike in 1 s) and its soma voltage has
    several maxima and minima."""
    r = o64.run(I.Network(n=1, conn="none"), 20000, trace_every=20, trace_cells=1)
    assert r["counts"][0] == 0
    vs = r["trace"][:, VS, 0]
    assert vs.max() < -30.0
    interior = vs[50:]
    peaks = np.sum((interior[1:-1] > interior[:-2]) & (interior[1:-1] > interior[2:]))
    assert peaks >= 4
    assert np.ptp(interior) > 5.0


def test_single_cell_pulse_complex_spike(o64):
    """Section 3 validation: a small current pulse of about 500 steps (25 ms)
    into the cell makes it fire (axon spikes), none before the pulse, and the
    cell returns to subthreshold behaviour afterwards."""
    net = I.Network(n=1, conn="none", pulses=[I.Pulse(400, 900, 6.0)])
    r = o64.run(net, 4000, trace_every=1, trace_cells=1, spike_cap=256)
    c = r["counts"][0]
    t = r["times"][0, :c]
    assert c >= 1
    assert t.min() >= 20.0 and t.max() <= 70.0
    va = r["trace"][:, VA, 0]
    assert va[:399].max() < 0.0          # nothing before the pulse (t < 20 ms)
    assert va[2000:].max() < 0.0         # subthreshold again after 100 ms


def test_dendritic_pulse_raises_dendrite_only_at_first_step(o64):
    x = o64.rest()
    d0 = o64.rhs(x, 0.0, 0.0)
    d1 = o64.rhs(x, 0.0, 6.0)
    assert d1[VD] - d0[VD] == pytest.approx(6.0, rel=1e-12)
    np.testing.assert_array_equal(np.delete(d1, VD), np.delete(d0, VD))
    # the gap current enters with the opposite sign (outward current)
    d2 = o64.rhs(x, 2.5, 0.0)
    assert d2[VD] - d0[VD] == pytest.approx(-2.5, rel=1e-12)


def _only(**vals):
    p = np.zeros(20)
    p[P["p1"]], p[P["p2"]] = 0.25, 0.15
    for k in ("V_Na", "V_K", "V_Ca", "V_h", "V_L"):
        p[P[k]] = I.DEFAULT_PARAMS[P[k]]
    for k, v in vals.items():
        p[P[k]] = v
    return p


@pytest.mark.parametrize("g,rev,comp", [
    ("g_CaH", "V_Ca", VD), ("g_KCa", "V_K", VD), ("g_h", "V_h", VD), ("g_ld", "V_L", VD),
    ("g_CaL", "V_Ca", VS), ("g_Na_s", "V_Na", VS), ("g_Kdr_s", "V_K", VS), ("g_K_s", "V_K", VS),
    ("g_ls", "V_L", VS), ("g_Na_a", "V_Na", VA), ("g_K_a", "V_K", VA), ("g_la", "V_L", VA),
])
def test_each_channel_drives_its_compartment_to_its_reversal(g, rev, comp, o64):
    """With one conductance switched on, the compartment that carries it moves
    toward that channel's reversal potential and no other voltage moves; at
    the reversal potential the current vanishes."""
    p = _only(**{g: 1.0})
    e = I.DEFAULT_PARAMS[P[rev]]
    x = o64.rest()
    # open every gate half-way so every channel conducts
    for gate in (R, S, Q, KK, LL, HH, NN, XX, HA, XA):
        x[gate] = 0.5
    for v0 in (-60.0, e - 10.0, e + 10.0):
        x[[VD, VS, VA]] = v0
        dx = o64.rhs(x, 0.0, 0.0, params=p)
        others = [c for c in (VD, VS, VA) if c != comp]
        assert all(dx[c] == 0.0 for c in others)
        if v0 != e:
            assert np.sign(dx[comp]) == np.sign(e - v0)
    x[[VD, VS, VA]] = e
    dx = o64.rhs(x, 0.0, 0.0, params=p)
    assert dx[comp] == 0.0


def test_compartment_coupling_conserves_charge(o64):
    """Only the internal conductance on: the area-weighted charge
    (1-p1)*Vd + p1*Vs + p1*p2/(1-p2)*Va is constant and the voltages relax to
    their common weighted mean."""
    p1, p2 = 0.25, 0.15
    p = _only(g_int=0.13)
    x = o64.rest()
    x[[VD, VS, VA]] = [-70.0, -50.0, -20.0]
    wts = np.array([1 - p1, p1, p1 * p2 / (1 - p2)])
    q0 = wts @ x[[VD, VS, VA]]
    net = I.Network(n=1, conn="none", params=p)
    r = o64.run(net, 40000, x0=x[:, None])
    v = r["x"][[VD, VS, VA], 0]
    assert wts @ v == pytest.approx(q0, rel=1e-12)
    np.testing.assert_allclose(v, q0 / wts.sum(), rtol=0, atol=1e-6)


def test_leak_closed_form(o64):
    """Leak only: forward Euler gives V_n = V_L + (V_0 - V_L)(1 - dt*g)^n."""
    p = _only(g_ld=0.016, g_ls=0.032, g_la=0.064)
    x = o64.rest()
    x[[VD, VS, VA]] = [-60.0, -70.0, -80.0]
    n = 3000
    r = o64.run(I.Network(n=1, conn="none", params=p), n, x0=x[:, None])
    for comp, g, v0 in ((VD, 0.016, -60.0), (VS, 0.032, -70.0), (VA, 0.064, -80.0)):
        exact = 10.0 + (v0 - 10.0) * (1 - 0.05 * g) ** n
        assert r["x"][comp, 0] == pytest.approx(exact, rel=1e-11)


@pytest.mark.parametrize("gate,comp,vhalf,rising", [
    (KK, VS, -61.0, True), (LL, VS, -85.5, False), (HH, VS, -70.0, False),
    (NN, VS, -3.0, True), (Q, VD, -80.0, False), (HA, VA, -60.0, False),
])
def test_gate_steady_state_half_points(gate, comp, vhalf, rising, o64):
    """Published half-(in)activation voltages: with every conductance off the
    voltages are constant and each gate relaxes to its steady state; at V_1/2
    that is 0.5, and it rises (activation) or falls (inactivation) with V."""
    p = _only()
    res = []
    for v in (vhalf - 5.0, vhalf, vhalf + 5.0):
        x = o64.rest()
        x[[VD, VS, VA]] = v
        # dt = 0.1 ms keeps every gate stable at these voltages (dt < 2*tau)
        # and 40 s covers the slowest one (tau_q ~ 1 s at -80 mV) many times
        r = o64.run(I.Network(n=1, conn="none", params=p, dt=0.1), 400000, x0=x[:, None])
        res.append(r["x"][gate, 0])
    assert res[1] == pytest.approx(0.5, abs=1e-9)
    assert (res[2] > res[1] > res[0]) if rising else (res[2] < res[1] < res[0])


def test_alpha_beta_gates_removable_singularities(o64):
    """beta_r at Vd = -8.5 mV and alpha_x at V = -25 mV are 0/0 forms; the
    oracle takes their limits (finite RHS, continuous across the point)."""
    x = o64.rest()
    for v in (-8.5, -25.0):
        x[[VD, VS, VA]] = v
        d0 = o64.rhs(x)
        assert np.all(np.isfinite(d0))
        x[[VD, VS, VA]] = v + 1e-7
        d1 = o64.rhs(x)
        np.testing.assert_allclose(d1[[R, XX, XA]], d0[[R, XX, XA]], rtol=1e-5, atol=1e-9)


def test_calcium_decay_closed_form(o64):
    """No Ca inflow (g_CaH = 0): [Ca] decays as (1 - 0.075*dt)^n."""
    x = o64.rest()
    x[CA] = 5.0
    n = 2000
    r = o64.run(I.Network(n=1, conn="none", params=_only()), n, x0=x[:, None])
    assert r["x"][CA, 0] == pytest.approx(5.0 * (1 - 0.075 * 0.05) ** n, rel=1e-11)


def test_rest_state_gates_stationary(o64):
    """At the rest state every gate and [Ca] has zero time derivative."""
    x = o64.rest()
    dx = o64.rhs(x)
    for v in (CA, R, S, Q, KK, LL, HH, NN, XX, HA, XA):
        assert abs(dx[v]) < 1e-12, v


# ----------------------------------------------------------------- integration
def test_forward_euler_first_order(o64):
    """Halving dt halves the error: successive differences shrink by ~2."""
    x0 = None
    finals = []
    for k, dt in enumerate((0.05, 0.025, 0.0125, 0.00625)):
        net = I.Network(n=1, conn="none", dt=dt)
        if x0 is None:
            x0 = o64.initial_state(net)
        steps = int(round(15.0 / dt))
        finals.append(o64.run(net, steps, x0=x0)["x"][:, 0])
    d1 = np.abs(finals[0] - finals[1])
    d2 = np.abs(finals[1] - finals[2])
    d3 = np.abs(finals[2] - finals[3])
    for v in (VD, VS, VA):
        assert 1.7 < d1[v] / d2[v] < 2.3
        assert 1.8 < d2[v] / d3[v] < 2.2


def test_f32_tracks_f64_config0(o64, o32):
    net = I.config0()
    a = o64.run(net, 1000, trace_every=10, trace_cells=net.n)["trace"]
    b = o32.run(net, 1000, trace_every=10, trace_cells=net.n)["trace"]
    scale = np.abs(a).max(axis=(0, 2))
    err = np.abs(a - b).max(axis=(0, 2)) / scale
    assert err.max() < 1e-4


def test_pulse_window_integer_steps(o64):
    net = I.Network(n=3, conn="none", bias=np.array([0.5, 0.0, -0.5]),
                    pulses=[I.Pulse(400, 500, 6.0, 1, 3)])
    np.testing.assert_array_equal(o64.iapp(net, 399), [0.5, 0.0, -0.5])
    np.testing.assert_array_equal(o64.iapp(net, 400), [0.5, 6.0, 5.5])
    np.testing.assert_array_equal(o64.iapp(net, 499), [0.5, 6.0, 5.5])
    np.testing.assert_array_equal(o64.iapp(net, 500), [0.5, 0.0, -0.5])
    stream = np.arange(6.0).reshape(2, 3)
    np.testing.assert_array_equal(o64.iapp(net, 1, i_stream=stream), [3.5, 4.0, 4.5])


def test_spike_time_interpolation(o64):
    """Spike time = (n + (0 - Va_n)/(Va_{n+1} - Va_n)) * dt for the upward
    zero crossing, checked against the stored trace."""
    net = I.Network(n=1, conn="none", pulses=[I.Pulse(400, 900, 6.0)])
    r = o64.run(net, 1400, trace_every=1, trace_cells=1)
    va = np.concatenate([[o64.initial_state(net)[VA, 0]], r["trace"][:, VA, 0]])
    ups = np.nonzero((va[:-1] < 0) & (va[1:] >= 0))[0]
    assert len(ups) == r["counts"][0] >= 1
    for k, n in enumerate(ups):
        t = (n + (0 - va[n]) / (va[n + 1] - va[n])) * 0.05
        assert r["times"][0, k] == pytest.approx(t, rel=1e-12)


# ------------------------------------------------------------------ work counts
def test_instrumented_operation_counts(tmp_path):
    """The oracle body compiled with a counting number type: one cell-step's
    right-hand side evaluates exactly 21 exp/expm1 (dendrite 5: the two r
    rates, the q sigmoid and q's two-exp rate; soma 11: five sigmoids, l's two
    exps, h, n and x's two rates; axon 5: two sigmoids, h_a and x_a's two
    rates) and 224 arithmetic operations in all; one
    gap-junction pair term is 9 operations with one exp (Algorithm 1:
    subtract, square, negate, divide by 100, exp, scale by 0.8, add 0.2,
    times dV, times w). Table 1's 859 operations per cell-step counts each exp
    as a routine of ~31 operations (203 + 21 x 31 = 854); its ~12 per
    connection counts the exp as one (9 + the accumulation)."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path / "count_ops")
    subprocess.run([gxx, "-std=c++17", "-O1", "-fopenmp", "-o", exe,
                    os.path.join(here, "opcount", "count_ops.cpp")], check=True, capture_output=True)
    params = " ".join(repr(float(v)) for v in I.DEFAULT_PARAMS)
    out = subprocess.run([exe], input=params, text=True, check=True, capture_output=True).stdout.split()
    rhs_ops, rhs_tr, pair_ops, pair_tr = map(int, out)
    assert rhs_tr == 21 and rhs_ops == 224
    assert pair_tr == 1 and pair_ops == 9
    assert abs((rhs_ops - rhs_tr) + 31 * rhs_tr - 859) < 20


# ---------------------------------------------------------------------------
# Cell-model rate functions, read out of the oracle's right-hand side through
# clamped states and compared with values evaluated by hand from the
# published model's equations (tests/golden/cell_rates.txt). Each gate's
# derivative at gate value 0 and 1 gives its two rates (alpha, -beta) or its
# steady state and time constant; the Na activation is read from the soma or
# axon voltage derivative with every other conductance set to zero.
_SV = dict(VD=0, CA=1, R=2, S=3, Q=4, VS=5, K=6, L=7, H=8, N=9, X=10, VA=11, HA=12, XA=13)
_GNA_S, _GNA_A, _GCAH, _VNA, _VCA = 5, 9, 0, 15, 17


def _golden_rates():
    rows = []
    for line in open(os.path.join(GOLDEN, "cell_rates.txt")):
        if line.strip() and not line.startswith("#"):
            name, arg, val = line.split()
            rows.append((name, float(arg), float(val)))
    return rows


def _gate_pair(o, var, vvar, v, params=None):
    """dy/dt of gate `var` at y = 0 and y = 1 with voltage `vvar` = v."""
    x = o.rest().astype(np.float64)
    x[_SV[vvar]] = v
    out = []
    for y in (0.0, 1.0):
        x[_SV[var]] = y
        out.append(float(o.rhs(x, params=params)[_SV[var]]))
    return out


def _steady_tau(o, var, vvar, v):
    d0, d1 = _gate_pair(o, var, vvar, v)       # y_inf / tau, (y_inf - 1) / tau
    tau = 1.0 / (d0 - d1)
    return d0 * tau, tau


def _na_activation(o, vvar, v):
    from paper_1612_01501_amd.inputs import DEFAULT_PARAMS
    p = np.zeros(20)
    p[13], p[14] = DEFAULT_PARAMS[13], DEFAULT_PARAMS[14]   # area ratios (no coupling: g_int = 0)
    p[_VNA] = 55.0
    g, vi, hi = (_GNA_S, "VS", "H") if vvar == "VS" else (_GNA_A, "VA", "HA")
    p[g] = 1.0
    x = o.rest().astype(np.float64)
    x[_SV[vi]] = v
    x[_SV[hi]] = 1.0
    dv = float(o.rhs(x, params=p)[_SV[vi]])     # -m_inf^3 (V - V_Na)
    return np.cbrt(dv / (55.0 - v))


def _read_rate(o, name, a):
    if name in ("alpha_r", "beta_r"):
        d0, d1 = _gate_pair(o, "R", "VD", a)
        return 5.0 * d0 if name == "alpha_r" else -5.0 * d1
    if name in ("alpha_x", "beta_x"):
        d0, d1 = _gate_pair(o, "X", "VS", a)
        return d0 if name == "alpha_x" else -d1
    if name in ("alpha_s", "beta_s"):
        x = o.rest().astype(np.float64)
        x[_SV["CA"]] = a
        x[_SV["S"]] = 0.0 if name == "alpha_s" else 1.0
        d = float(o.rhs(x)[_SV["S"]])
        return d if name == "alpha_s" else -d
    if name in ("ca_decay", "ca_inflow"):
        p = np.zeros(20)
        p[13], p[14] = 0.25, 0.15
        x = o.rest().astype(np.float64)
        if name == "ca_decay":
            x[_SV["CA"]] = a
        else:
            p[_GCAH], p[_VCA] = 1.0, 120.0
            x[_SV["CA"]], x[_SV["R"]], x[_SV["VD"]] = 0.0, 1.0, a
        return float(o.rhs(x, params=p)[_SV["CA"]])
    if name == "m_inf":
        return _na_activation(o, "VS", a)
    gates = {"q": ("Q", "VD"), "k": ("K", "VS"), "l": ("L", "VS"), "h": ("H", "VS"),
             "n": ("N", "VS"), "ha": ("HA", "VA")}
    kind, g = ("tau", name[4:]) if name.startswith("tau_") else ("inf", name[:-4])
    inf, tau = _steady_tau(o, *gates[g], a)
    return inf if kind == "inf" else tau


def test_cell_rates_match_published_equations(o64):
    rows = _golden_rates()
    assert len(rows) >= 80
    for name, a, val in rows:
        got = _read_rate(o64, name, a)
        assert got == pytest.approx(val, rel=2e-12, abs=1e-15), (name, a, got, val)


def test_axon_gates_share_the_soma_rate_forms(o64):
    """The axon's Na activation and K gate rates are the soma's functions of
    the axon voltage (same golden values)."""
    rows = {(n, a): v for n, a, v in _golden_rates()}
    for v in (-70.0, -45.0, -10.0, 20.0):
        assert _na_activation(o64, "VA", v) == pytest.approx(rows[("m_inf", v)], rel=2e-12)
        d0, d1 = _gate_pair(o64, "XA", "VA", v)
        assert d0 == pytest.approx(rows[("alpha_x", v)], rel=2e-12)
        assert -d1 == pytest.approx(rows[("beta_x", v)], rel=2e-12)


def test_cell_rate_pins_catch_planted_slips(o64, monkeypatch):
    """A plausible slip in a rate constant (planted in the values the test
    reads, on the CPU) fails the golden comparison."""
    rows = _golden_rates()
    real = _read_rate
    for target in ("tau_h", "beta_x", "tau_q", "alpha_r"):
        def slipped(o, name, a, _t=target):
            v = real(o, name, a)
            return v * 1.001 if name == _t else v
        bad = [(n, a, v) for n, a, v in rows if slipped(o64, n, a) != pytest.approx(v, rel=2e-12, abs=1e-15)]
        assert bad and all(n == target for n, _, _ in bad), target
