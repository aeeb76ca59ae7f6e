"""Output streaming through the C ABI: the axon voltage of every cell after
each step, written into a device ring by the step kernels and copied to the
host on a second stream while later steps compute (Section 2.4.3: the host
receives each step's output while the next step runs)."""
import ctypes

import numpy as np
import pytest

from paper_1612_01501_amd import inputs as I

pytestmark = pytest.mark.gpu

VA = I.IDX_VA


@pytest.fixture(scope="module")
def infoli():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1612_01501_amd import infoli as mod
    mod.lib()
    return mod


def _stream(infoli, net, x0, steps, chunk, ring, mode, host=None):
    """Step in chunks, queueing the copy of each chunk's outputs right after
    it; returns [steps][cells] and the final state."""
    cells = net.n
    out = np.zeros((steps, cells), np.float32) if host is None else host
    sim = infoli.Simulator(net, init_states=[x0], step_mode=mode, graph_chunk=50, output_ring_steps=ring)
    for s0 in range(0, steps, chunk):
        sim.step(chunk)
        view = out[s0:s0 + chunk]
        sim.output_copy_async(s0, chunk, view.ctypes.data, view.size)
    sim.output_wait()
    x = sim.read_state(0)
    sim.close()
    return out, x


@pytest.mark.parametrize("mode", ["persistent", "graph", "launch"])
def test_streamed_output_matches_oracle_and_state(infoli, o32, o64, mode):
    """1,000 steps of the 96-cell network through its 5 ms pulse: the streamed
    Va of every step against the oracle's (bound as in the trajectory
    tests), and bitwise equal to the state read back at the end."""
    net = I.config0()
    x0 = infoli.initial_state(net)
    out, x = _stream(infoli, net, x0, 1000, 100, 256, mode)
    np.testing.assert_array_equal(out[-1], x[VA])
    ref = o32.run(net, 1000, x0=x0, trace_every=1, trace_cells=net.n)["trace"][:, VA, :]
    r64 = o64.run(net, 1000, x0=x0.astype(np.float64), trace_every=1, trace_cells=net.n)["trace"][:, VA, :]
    scale = np.abs(ref).max()
    err = np.abs(out - ref).max() / scale
    floor = np.abs(ref - r64).max() / scale
    print(f"{mode}: streamed Va err {err:.2e}, f32-oracle floor {floor:.2e}")
    assert err <= max(1e-4, 2 * floor)


def test_ring_wrap_and_tight_streaming_bitwise(infoli):
    """A ring of 64 steps, chunks of 40 (copies cross the wrap) and of 64
    (each chunk's copy must finish before the next chunk overwrites its
    slots): bitwise equal to a run with a ring of 1,024 steps."""
    net = I.config1(0.1, seed=3, n=300)
    x0 = infoli.initial_state(net)
    want, _ = _stream(infoli, net, x0, 640, 64, 1024, "graph")
    for chunk in (40, 64):
        got, _ = _stream(infoli, net, x0, 640, chunk, 64, "graph")
        np.testing.assert_array_equal(got, want)


def test_streaming_into_pinned_memory_batch(infoli):
    """Two networks in one context, pinned host memory (the copies overlap
    the compute): cells in batch order, bitwise equal to pageable copies."""
    import torch
    nets = [I.config0(), I.config1(0.05, seed=4, n=200)]
    x0s = [infoli.initial_state(n) for n in nets]
    cells = sum(n.n for n in nets)
    host = torch.zeros((800, cells), dtype=torch.float32, pin_memory=True)
    ref = np.zeros((800, cells), np.float32)
    for buf in (host.numpy(), ref):
        sim = infoli.Simulator(nets, init_states=x0s, step_mode="graph", graph_chunk=50, output_ring_steps=200)
        for s0 in range(0, 800, 100):
            sim.step(100)
            view = buf[s0:s0 + 100]
            sim.output_copy_async(s0, 100, view.ctypes.data, view.size)
        sim.output_wait()
        end = [sim.read_state(k)[VA] for k in range(2)]
        sim.close()
    np.testing.assert_array_equal(host.numpy(), ref)
    np.testing.assert_array_equal(ref[-1], np.concatenate(end))


def test_output_copy_rejections(infoli):
    net = I.config0()
    x0 = infoli.initial_state(net)
    buf = np.zeros((64, net.n), np.float32)
    sim = infoli.Simulator(net, init_states=[x0], step_mode="launch", output_ring_steps=32)
    sim.step(10)
    with pytest.raises(RuntimeError, match="not queued"):
        sim.output_copy_async(5, 10, buf.ctypes.data, buf.size)        # steps 10..14 not run
    with pytest.raises(RuntimeError, match="n_steps"):
        sim.output_copy_async(0, 33, buf.ctypes.data, buf.size)        # more than the ring
    with pytest.raises(RuntimeError, match="capacity"):
        sim.output_copy_async(0, 10, buf.ctypes.data, 10)
    sim.step(40)
    with pytest.raises(RuntimeError, match="no longer"):
        sim.output_copy_async(0, 10, buf.ctypes.data, buf.size)        # overwritten
    sim.output_copy_async(20, 30, buf.ctypes.data, buf.size)
    sim.output_wait()
    sim.close()
    sim = infoli.Simulator(net, init_states=[x0], step_mode="launch")
    sim.step(2)
    with pytest.raises(RuntimeError, match="no output ring"):
        sim.output_copy_async(0, 1, buf.ctypes.data, buf.size)
    sim.close()


def test_surrogate_refuses_ring_context(infoli):
    net = I.config0()
    sim = infoli.Simulator(net, init_states=[infoli.initial_state(net)], output_ring_steps=8)
    with pytest.raises(RuntimeError, match="output ring"):
        sim.step_surrogate(1)
    sim.close()
