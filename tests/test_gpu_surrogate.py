"""The learned surrogate on the GPU: its MLP kernels against the numpy oracle
(emulated BF16 at the same rounding points), the drift check and plain
fallback, the held-gap plain macro step against the CPU oracle, and the
trained surrogate against the plain method (accuracy and speed)."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_1612_01501_amd import inputs as I

pytestmark = pytest.mark.gpu

VD, VS, VA = 0, 5, 11


@pytest.fixture(scope="module")
def infoli():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1612_01501_amd import infoli as mod
    mod.lib()
    return mod


def _params(seed):
    w = I.mlp_init_params(seed).astype(np.float64)
    w += I.rng(seed + 1).normal(0.0, 0.02, w.shape)          # non-zero biases
    return w.astype(np.float32)


# ------------------------------------------------------------------ kernels vs oracle
@pytest.mark.parametrize("batch", [16, 64, 1024])
def test_mlp_forward_matches_oracle(infoli, batch):
    w = _params(3)
    x, _ = I.mlp_batch(batch, 4)
    y = infoli.mlp_forward(w, x).astype(np.float64)
    ref, _ = M.forward(w.astype(np.float64), x, bf16=True)
    err = np.abs(y - ref) / (1.0 + np.abs(ref))
    print(f"forward B={batch}: max scaled error {err.max():.2e}")
    assert err.max() <= 2e-3


@pytest.mark.parametrize("batch", [64, 4096])
def test_mlp_gradients_match_oracle(infoli, batch):
    """GPU loss and gradients against the emulated-BF16 oracle, element by
    element: |g - g_ref| <= 1e-3 x the largest |g_ref| of the element's
    parameter block (the scale floor: BF16 rounding points that fp32 and
    fp64 sums send different ways move single elements by up to ~1e-4 of
    that scale), and the 2-norm of each block's error <= 1e-3 of its own."""
    w = _params(5)
    x, t = I.mlp_batch(batch, 6)
    loss, g = infoli.mlp_loss_grad(w, x, t)
    rl, rg = M.loss_and_grad(w.astype(np.float64), x, t, bf16=True)
    assert loss == pytest.approx(rl, rel=1e-4)
    gp, rp = M.unpack(g.astype(np.float64)), M.unpack(rg)
    worst = worst_el = 0.0
    for name, _ in M.SHAPES:
        a, b = gp[name], rp[name]
        if name in ("W3", "b3"):                    # rows 14, 15 are padding outputs
            assert np.all(a[14:] == 0), name
            a, b = a[:14], b[:14]
        scale = np.abs(b).max()
        assert scale > 0, name
        el = np.abs(a - b) / scale
        worst_el = max(worst_el, float(el.max()))
        assert np.all(el <= 1e-3), (name, np.unravel_index(np.argmax(el), el.shape), el.max())
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        worst = max(worst, rel)
        assert rel <= 1e-3, (name, rel)
    print(f"gradients B={batch}: worst element error / block scale {worst_el:.2e}, "
          f"worst block relative error {worst:.2e}")


def _bf16_other(v):
    """For float32 values v, the BF16 value on the far side of v from its
    nearest BF16 value (the one a rounding tie can go to instead)."""
    r = M.bf16_round(v)
    u = r.view(np.uint32).astype(np.int64)
    away = np.abs(v) > np.abs(r)
    o = np.where(away, u + 0x10000, u - 0x10000).astype(np.uint32)
    return r, o.view(np.float32)


def test_surrogate_candidates_match_oracle(infoli, o32):
    """One macro step in which no cell is checked and every cell passes the
    guards, so each cell takes its MLP candidate x + out_std * y + out_mean,
    y = MLP((feature - in_mean) * in_rstd) over the 14 states, the gap current
    and the evoked input. Compared element by element with the oracle MLP
    (emulated BF16) fed the fp32 oracle's state, gap current and input, on
    1,000 cells (a ragged last wave) of a 50-degree network. Distinct
    per-feature normalisation constants make a permuted feature or output
    fail. The GPU's gap current differs from the oracle's by up to the fp32
    gap bound; where that can move the BF16 rounding of the normalised gap
    feature (the oracle's value within that distance of a rounding tie) the
    candidate may match the oracle at either BF16 neighbour."""
    from test_gpu_parity import gap_bound
    net = I.config4(seed=3, n=1000, degree=50.0)
    xs = o32.run(net, 60)["x"]                        # gates spread by the jitter
    ig = o32.gap(net, xs[VD])
    ia = o32.iapp(net, 0)
    feats = np.concatenate([xs, ig[None], ia[None]]).T.astype(np.float32)      # [n][16]
    mean = feats.astype(np.float64).mean(axis=0)
    std = feats.astype(np.float64).std(axis=0)
    rstd = 1.0 / np.maximum(std, 1e-3 * np.maximum(np.abs(mean), 1.0))
    k = np.arange(16)
    out_mean = 1e-3 * (k - 7.5)
    out_std = 0.01 * (1.0 + 0.25 * k)
    norm = np.concatenate([mean, rstd, out_mean, out_std]).astype(np.float32)
    w = _params(11)

    sim = infoli.Simulator(net, init_states=[xs], step_mode="graph")
    sim.surrogate_set(w, norm)
    r = sim.step_surrogate(1, mode="mlp", sample_every=0)
    got = sim.read_state(0).astype(np.float64).T                             # [n][14]
    sim.close()
    assert r["checked"] == 0 and r["guarded"] == 0 and r["plain_cell_macro_steps"] == 0, r

    f32 = np.float32
    nm, nr = norm[:16], norm[16:32]
    xn = ((feats - nm) * nr).astype(np.float32)        # the kernel's order: (raw - mean) * rstd
    wd = w.astype(np.float64)

    def candidate(xin):
        y, _ = M.forward(wd, xin, bf16=True)
        return y, xs.T.astype(np.float64) + (y[:, :14] * norm[48:62] + norm[32:46])

    y, ref = candidate(xn)
    tol = 2e-3 * (1.0 + np.abs(y[:, :14])) * norm[48:62] + 2 * np.finfo(f32).eps * np.abs(ref)
    ok = np.abs(got - ref) <= tol
    # the gap feature near a BF16 rounding tie: either neighbour
    r14, o14 = _bf16_other(xn[:, 14])
    mid = 0.5 * (r14.astype(np.float64) + o14)
    near = np.abs(xn[:, 14] - mid) <= 1.01 * gap_bound(net, xs[VD]) * nr[14] + 4 * np.finfo(f32).eps * np.abs(mid)
    alt = xn.copy()
    alt[:, 14] = o14
    y2, ref2 = candidate(alt)
    ok2 = np.abs(got - ref2) <= 2e-3 * (1.0 + np.abs(y2[:, :14])) * norm[48:62] + 2 * np.finfo(f32).eps * np.abs(ref2)
    cell_ok = np.all(ok, axis=1) | (near & np.all(ok2, axis=1))
    bad = np.nonzero(~cell_ok)[0]
    err = (np.abs(got - ref) / tol).max()
    print(f"surrogate candidates: max error / bound {err:.2e}, {int(near.sum())} cells near a gap-feature tie")
    assert bad.size == 0, (bad[:8], (np.abs(got - ref) / tol)[bad[:8]].max(axis=1))
    # the step moved every cell by its MLP increment (not a copy of the state)
    assert np.all(np.any(got != xs.T, axis=1))


def test_adam_step_matches_oracle(infoli):
    rs = I.rng(9)
    w = rs.normal(0, 0.1, M.N_PARAMS).astype(np.float32)
    m = rs.normal(0, 0.01, M.N_PARAMS).astype(np.float32)
    v = np.abs(rs.normal(0, 0.001, M.N_PARAMS)).astype(np.float32)
    g = rs.normal(0, 0.05, M.N_PARAMS).astype(np.float32)
    w1, m1, v1 = infoli.mlp_adam_step(w, m, v, g, 7, lr=2e-3)
    rw, rm, rv = M.adam_step(w.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                             g.astype(np.float64), 7, lr=2e-3)
    np.testing.assert_allclose(m1, rm, rtol=1e-5, atol=2e-8)
    np.testing.assert_allclose(v1, rv, rtol=3e-5, atol=1e-12)
    np.testing.assert_allclose(w1, rw, rtol=1e-5, atol=2e-7)


# ------------------------------------------------------------------ held-gap macro step
def test_plain_hold_matches_oracle(infoli, o32):
    """Macro steps without the MLP: the gap current from the macro step's
    starting Vd held for four plain steps; compared with the same scheme built
    from the oracle's gap and right-hand-side functions."""
    net = I.Network(n=64, conn="uniform", g=0.04, jitter=I.voltage_jitter(64, 21),
                    bias=I.input_bias(64, 22), pulses=[I.Pulse(40, 140, 6.0)])
    x0 = infoli.initial_state(net)
    sim = infoli.Simulator(net, init_states=[x0], step_mode="graph")
    sim.step_surrogate(50, mode="plain_hold")
    got = sim.read_state(0)
    sim.close()
    x = x0.copy()
    P = net.params
    for m in range(50):
        ig = o32.gap(net, x[VD])
        for k in range(4):
            ia = o32.iapp(net, 4 * m + k)
            for i in range(net.n):
                x[:, i] = x[:, i] + np.float32(net.dt) * o32.rhs(x[:, i], ig[i], ia[i], P)
    scale = np.abs(x).max(axis=1)
    err = (np.abs(got.astype(np.float64) - x) .max(axis=1) / scale).max()
    assert err <= 1e-4, err


# ------------------------------------------------------------------ drift check and fallback
def _trained(infoli, net, x0, **cfg):
    sim = infoli.Simulator(net, init_states=[x0], step_mode="graph")
    rep, hist = sim.surrogate_train(I.mlp_init_params(5000), **cfg)
    return sim, rep, hist


def test_forced_fallback(infoli):
    """theta = 0: every checked cell is flagged and held on the plain method;
    checking every cell with theta = inf gives exactly the plain result."""
    net = I.config4(seed=2, n=4096, degree=200)
    x0 = infoli.initial_state(net)
    sim, rep, _ = _trained(infoli, net, x0, steps=200, n_transitions=100_000)
    params, norm = sim.surrogate_get()
    r1 = sim.step_surrogate(1, theta_mv=0.0, sample_every=64, hold_steps=3)
    expected = sum(1 for c in range(net.n) if (c + sim.info()["step"] // 4 - 1) % 64 == 0)
    assert r1["checked"] == expected and r1["flagged"] == expected
    r2 = sim.step_surrogate(1, theta_mv=0.0, sample_every=64, hold_steps=3)
    assert r2["plain_cell_macro_steps"] >= expected + r2["checked"]
    sim.close()
    out = []
    for mode, kw in (("mlp", dict(theta_mv=1e30, sample_every=1)), ("plain_hold", {})):
        s = infoli.Simulator(net, init_states=[x0], step_mode="graph")
        s.surrogate_set(params, norm)
        r = s.step_surrogate(10, mode=mode, **kw)
        out.append(s.read_state(0))
        s.close()
        if mode == "mlp":
            assert r["checked"] == 10 * net.n and r["flagged"] == 0
    np.testing.assert_array_equal(out[0], out[1])


def test_guards_send_cells_to_plain(infoli):
    """Cells outside the MLP's regime (a voltage above v_max, [Ca] above
    ca_max) take the plain method: with no sampled checks their macro step
    equals the held-gap plain step bit for bit, and each is counted as
    guarded; cells inside the regime and away from it take the MLP."""
    net = I.config4(seed=4, n=2048, degree=100)
    x0 = infoli.initial_state(net)
    odd = {10: (VS, -30.0), 20: (1, 50.0), 30: (VD, -35.0), 40: (VA, -20.0)}
    for i, (v, val) in odd.items():
        x0[v, i] = val
    sim, _, _ = _trained(infoli, net, x0, steps=200, n_transitions=100_000)
    params, norm = sim.surrogate_get()
    sim.close()
    out, reps = {}, {}
    for mode in ("mlp", "plain_hold"):
        s = infoli.Simulator(net, init_states=[x0], step_mode="graph")
        s.surrogate_set(params, norm)
        reps[mode] = s.step_surrogate(1, mode=mode, sample_every=0)
        out[mode] = s.read_state(0)
        s.close()
    r = reps["mlp"]
    assert r["checked"] == 0 and r["guarded"] >= len(odd)
    assert r["plain_cell_macro_steps"] == r["guarded"]
    for i in odd:
        np.testing.assert_array_equal(out["mlp"][:, i], out["plain_hold"][:, i])
    differs = np.any(out["mlp"] != out["plain_hold"], axis=0)
    assert differs.sum() >= net.n - r["guarded"] - 16     # the rest took the MLP


def test_surrogate_set_get_roundtrip_and_errors(infoli):
    net = I.Network(n=100, conn="none")
    sim = infoli.Simulator(net)
    with pytest.raises(infoli.InfoliError) as e:
        sim.step_surrogate(1)
    assert e.value.status == 6                     # no surrogate yet
    w = _params(1)
    norm = np.concatenate([np.zeros(16), np.ones(16), np.zeros(16), np.ones(16)]).astype(np.float32)
    bad = norm.copy()
    bad[20] = 0.0
    with pytest.raises(infoli.InfoliError):
        sim.surrogate_set(w, bad)
    sim.surrogate_set(w, norm)
    w2, n2 = sim.surrogate_get()
    np.testing.assert_array_equal(w2, w)
    np.testing.assert_array_equal(n2, norm)
    sim.close()


# ------------------------------------------------------------------ trained surrogate vs plain
def test_trained_surrogate_accuracy_and_gain(infoli):
    """The 65,536-cell recipe at 8,192 cells (mean degree 1,000, g = 3.84e-3,
    bias, pulse, jitter): after training on device-generated transitions the
    surrogate run stays within 1 mV RMSE of the plain run over 2,000 steps,
    spikes (if any) within 0.5 ms, and it is faster than the plain method
    (drift checks on, default guards)."""
    net = I.config4(seed=1, n=8192)
    x0 = infoli.initial_state(net)
    sim, rep, hist = _trained(infoli, net, x0)        # defaults: 10^6 transitions, 20,000 steps
    print(f"training: {rep['n_transitions']} transitions, loss {rep['loss_first']:.3e} -> "
          f"{rep['loss_last']:.3e}, data {rep['data_ms']:.1f} ms, train {rep['train_ms']:.1f} ms")
    assert rep["loss_last"] < 0.01 * rep["loss_first"]
    params, norm = sim.surrogate_get()
    sim.close()

    plain = infoli.Simulator(net, init_states=[x0], step_mode="graph", graph_chunk=100)
    surr = infoli.Simulator(net, init_states=[x0], step_mode="graph", graph_chunk=100)
    surr.surrogate_set(params, norm)
    t_plain = t_surr = 0.0
    sq, cnt = 0.0, 0
    for _ in range(10):
        plain.step(200)
        plain.sync()
        t_plain += plain.last_step_ms()
        r = surr.step_surrogate(50)
        t_surr += r["ms"]
        a, b = plain.read_state(0), surr.read_state(0)
        d = (a[[VD, VS, VA]] - b[[VD, VS, VA]]).astype(np.float64)
        sq += float((d * d).sum())
        cnt += d.size
    rmse = np.sqrt(sq / cnt)
    ca, ta = plain.read_spikes(0)
    cb, tb = surr.read_spikes(0)
    plain.close()
    surr.close()
    print(f"surrogate vs plain over 2,000 steps: voltage RMSE {rmse:.3f} mV, "
          f"plain {t_plain:.2f} ms, surrogate {t_surr:.2f} ms, speedup {t_plain / t_surr:.2f}x, "
          f"spikes plain {ca.sum()} surrogate {cb.sum()}")
    assert rmse <= 1.0
    assert np.all(np.abs(ca.astype(np.int64) - cb) <= 1)
    for i in np.nonzero((ca > 0) & (cb > 0))[0][:200]:
        k = min(ca[i], cb[i], ta.shape[1])
        assert np.max(np.abs(np.sort(ta[i, :k]) - np.sort(tb[i, :k]))) <= 0.5
    assert t_surr < t_plain


def test_mlp_gain_over_held_gap(infoli):
    """What the learned part gains over the same macro step without it (the
    gap current held for four plain steps), at 65,536 cells of mean degree
    1,000: both macro steps, and the plain method, timed on the device over
    500 macro steps (2,000 dt) after a warm-up. Printed: each one's device
    time per 4 dt and the two gains. Asserted: the surrogate beats the plain
    method, and the held-gap step (gap current once per 4 dt, four exact cell
    updates) beats the MLP step: a cell's MLP evaluation (41k MFMA flops,
    256 SiLU activations, guards, the drift re-check of 1/64 cells) costs
    more than four exact cell updates, and the gap current, which both
    compute once per macro step, is most of either step."""
    net = I.config4()
    x0 = infoli.initial_state(net)
    sim, rep, _ = _trained(infoli, net, x0)
    params, norm = sim.surrogate_get()
    sim.close()
    per4 = {}
    for mode in ("mlp", "plain_hold"):
        s = infoli.Simulator(net, init_states=[x0], step_mode="graph")
        s.surrogate_set(params, norm)
        s.step_surrogate(25, mode=mode)
        ms = sum(s.step_surrogate(50, mode=mode)["ms"] for _ in range(10))
        per4[mode] = ms / 500
        s.close()
    plain = infoli.Simulator(net, init_states=[x0], step_mode="graph", graph_chunk=100)
    plain.step(100)
    plain.sync()
    ms = 0.0
    for _ in range(10):
        plain.step(200)
        plain.sync()
        ms += plain.last_step_ms()
    plain.close()
    per4["plain"] = ms / 500
    gain_plain = per4["plain"] / per4["mlp"]
    gain_hold = per4["plain_hold"] / per4["mlp"]
    print(f"per 4 dt at 65,536 cells: plain {per4['plain'] * 1e3:.1f} us, held gap {per4['plain_hold'] * 1e3:.1f} us, "
          f"MLP {per4['mlp'] * 1e3:.1f} us; surrogate vs plain {gain_plain:.2f}x, "
          f"MLP gain over held gap {gain_hold:.2f}x")
    assert gain_plain > 1.0
    assert gain_hold < 1.0, "the MLP step now beats the held-gap step: the design's reading of the gain is out of date"
