#!/usr/bin/env python3
"""Throughput of the InfOli step on one MI355X.

A "step" advances every network of the workload by one synchronous time step
(dt = 0.05 ms): gap-junction currents plus the three-compartment update of
every cell, all in the library's HIP kernels. Inputs are synthetic (seeded),
shaped like the paper's networks, and resident in device memory before the
timed region starts.

Workloads (--workload):
  csr4096  three 4,096-cell symmetric Erdos-Renyi CSR networks at 1 %, 10 %
           and 50 % density (g = 0.04, bias N(0, 0.5), 6 uA/cm^2 pulse at
           20-25 ms), stepped together: the default, 20,000 steps
  uni96    96 cells all-to-all (g = 0.04), 2,000 steps
  uni16k   16,384 cells all-to-all (g = 0.04*96/N), 4,000 steps
  surr65k  65,536 cells, symmetric ER graph of mean degree 1,000 (CSR,
           g = 3.84e-3), bias, pulse, jitter: the plain method for 10,000
           steps against the trained MLP surrogate for 2,500 macro steps of
           4 dt (drift check 1/64 cells, theta 0.5 mV), with the two
           ablations (held gap without MLP; MLP without fallback)
  csr65k   the surr65k network stepped by the plain method only, 2,000
           steps (the large-CSR, column-blocked gap path)
  ngj16m   2^24 uncoupled cells: the compartment update alone, 1.95 GB of
           state per step (beyond the 256 MB cache), 200 steps
  valid120k the paper's validation run: 96 cells, 25 ms pulse, 120,000 steps
           (6 s) with every step's axon voltages streamed to the host
  sgj65k   the csr65k network with simplified gap junctions (w * dV), 2,000
           steps
  sgj16k   the uni16k network with simplified gap junctions (the closed
           form g (N Vd_i - sum Vd)), 4,000 steps
  batch256 256 independent networks, N_k ~ U{64..2048}, density ~ U{5, 25,
           100 %} (100 % all-to-all, else ER CSR), g_k ~ U[0.01, 0.08],
           pulse amplitude ~ U[2, 10] uA/cm^2, 10,000 steps, one launch per
           step replayed from a HIP graph

Prints one JSON line (rank 0) with the throughput, a roofline entry for the
step kernel and the CPU oracle timed on a bounded sample of the same work.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_1612_01501_amd import inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0

# Measured HBM traffic of the step kernel per workload (rocprofv3 FETCH_SIZE
# and WRITE_SIZE, scaled by a plain-copy calibration), valid only for the
# kernel sources it was taken with.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
KERNEL_SOURCES = ("paper_1612_01501_amd/csrc/step_kernel.hpp", "paper_1612_01501_amd/csrc/cell_model.hpp",
                  "paper_1612_01501_amd/csrc/runtime.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """Bytes per launch, or None when no counters were taken for this
    workload or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            entry = json.load(fh).get(workload)
    except (OSError, ValueError):
        return None
    if not entry or entry.get("kernel_sources_sha256") != kernel_source_hash():
        return None
    return entry["bytes_per_launch"]
WORKLOADS = {
    "csr4096": dict(steps=20000, warmup=1000),
    "uni96": dict(steps=2000, warmup=200),
    "uni16k": dict(steps=4000, warmup=100),
    "batch256": dict(steps=10000, warmup=200),
    "surr65k": dict(steps=10000, warmup=100),
    "csr65k": dict(steps=2000, warmup=100),
    "ngj16m": dict(steps=200, warmup=10),
    "valid120k": dict(steps=120000, warmup=1000),
    "sgj65k": dict(steps=2000, warmup=100),
    "sgj16k": dict(steps=4000, warmup=200),
}


def build_workload(name):
    if name == "csr4096":
        nets = [I.config1(p) for p in (0.01, 0.1, 0.5)]
        desc = ("3 x 4,096-cell symmetric Erdos-Renyi gap graphs (1/10/50 % density) as CSR, "
                "g=0.04 mS/cm^2, bias N(0,0.5), 6 uA/cm^2 pulse steps [400,500), +-1 mV jitter, FP32, dt=0.05 ms")
    elif name == "uni96":
        nets = [I.config0()]
        desc = "96 cells all-to-all, g=0.04 mS/cm^2, 6 uA/cm^2 pulse steps [400,500), +-1 mV jitter, FP32, dt=0.05 ms"
    elif name == "batch256":
        nets = I.config3()
        desc = ("256 networks, N_k ~ U{64..2048}, density ~ U{5,25,100 %} (100 % all-to-all, else ER CSR), "
                "g_k ~ U[0.01,0.08] mS/cm^2, pulse A_k ~ U[2,10] uA/cm^2 steps [400,500), +-1 mV jitter, FP32, dt=0.05 ms")
    elif name == "surr65k":
        nets = [I.config4()]
        desc = ("65,536 cells, symmetric ER gap graph of mean degree 1,000 (CSR), g=3.84e-3 mS/cm^2, "
                "bias N(0,0.5), 6 uA/cm^2 pulse steps [400,500), +-1 mV jitter, FP32, dt=0.05 ms; "
                "MLP 16-128-128-16 BF16 on MFMA, 4 dt per macro step")
    elif name == "csr65k":
        nets = [I.config4()]
        desc = ("65,536 cells, symmetric ER gap graph of mean degree 1,000 (CSR), g=3.84e-3 mS/cm^2, "
                "bias N(0,0.5), 6 uA/cm^2 pulse steps [400,500), +-1 mV jitter, FP32, dt=0.05 ms; plain method")
    elif name == "valid120k":
        nets = [I.config0()]
        nets[0].pulses = [I.Pulse(400, 900, 6.0)]
        desc = ("the paper's validation run: 96 cells all-to-all, g=0.04 mS/cm^2, jitter, 25 ms pulse of "
                "6 uA/cm^2 at t=20 ms, 120,000 steps (6 s), the axon voltage of every cell streamed to "
                "pinned host memory every 1,000 steps while later steps compute")
    elif name == "sgj65k":
        nets = [I.config4()]
        nets[0].gap = "sgj"
        desc = ("65,536 cells, symmetric ER graph of mean degree 1,000 (CSR), simplified gap junctions "
                "w*dV, g=3.84e-3 mS/cm^2, bias N(0,0.5), pulse, jitter, FP32, dt=0.05 ms")
    elif name == "sgj16k":
        nets = [I.config2()]
        nets[0].gap = "sgj"
        desc = ("16,384 cells all-to-all, simplified gap junctions w*dV (closed form g*(N*Vd_i - sum Vd)), "
                "g=0.04*96/N mS/cm^2, +-1 mV jitter, no input, FP32, dt=0.05 ms")
    elif name == "ngj16m":
        n = 1 << 24
        nets = [I.Network(n=n, conn="none", jitter=I.voltage_jitter(n, 2000), bias=I.input_bias(n, 3000),
                          pulses=[I.Pulse(400, 500, 6.0)], label="ngj_n16m")]
        desc = ("16,777,216 uncoupled cells (no gap junctions: the compartment update alone, 1.95 GB of "
                "state per step, beyond the 256 MB cache), bias N(0,0.5), jitter, FP32, dt=0.05 ms")
    elif name == "uni16k":
        nets = [I.config2()]
        desc = "16,384 cells all-to-all, g=0.04*96/N mS/cm^2, +-1 mV jitter, no input, FP32, dt=0.05 ms"
    else:
        raise SystemExit(f"unknown workload {name}")
    return nets, desc


# Uniform all-to-all kernel: per directed pair one v_sub, one v_mul, one
# v_exp_f32 and one v_fma (w = g factored out, the linear 0.2*dV part in
# closed form). Full-rate VALU ops cost 1 lane-slot; v_exp_f32 issues at half
# rate on gfx950 (a register-only loop measures 16.3 T exp/s against 34.1 T
# fma/s), so it costs EXP_SLOTS = 2. 256 CUs x 64 lanes x 2.4 GHz.
LANE_SLOTS_PER_S = 256 * 64 * 2.4e9
EXP_SLOTS = 2
UNIFORM_SLOTS_PER_PAIR = 3 + EXP_SLOTS
# Compartment update per cell-step: 278 VALU instructions in its compiled
# form, of which 39 transcendental (21 v_exp_f32, 18 v_rcp_f32) at half rate,
# costing a second slot each.
CELL_SLOTS = 278 + 39


def algorithmic_bytes(nets, paths=None):
    """Bytes one step launch must move at minimum, in the format each network
    is streamed in (`paths`: the library's gap path per network; None takes
    the CSR gather format): per cell 14 state floats in and out plus the bias
    (116 B); per CSR edge its column (uint16 when every CSR network has
    <= 65,536 cells, else int32) plus its fp32 weight when the network has
    per-edge weights, and per CSR row its row pointer (8 B); for a network on
    the coupling bitmap instead, one bit per (row, column) pair in rows of
    whole 32-bit words. Gathered neighbour voltages are cache hits and not
    counted."""
    col_b = 2 if all(n.n <= 65536 for n in nets if n.conn == "csr") else 4
    b = 0
    for k, n in enumerate(nets):
        b += 116 * n.n
        if n.conn == "csr" and paths is not None and paths[k] == "csr_bitmap":
            b += 4 * n.n * ((n.n + 31) // 32)
        elif n.conn == "csr":
            b += (col_b + (4 if n.w_csr is not None else 0)) * int(n.row_ptr[-1]) + 8 * n.n
        elif n.conn == "dense":
            b += 4 * n.n * n.n
    return b


# CSR edge: v_sub, v_mul, v_mul, v_exp_f32 (2 slots), v_fma, v_add and two
# address operations for the 16-bit column gather.
CSR_SLOTS_PER_EDGE = 9
# Simplified gap junctions, per CSR edge: v_sub, v_fma and the two address
# operations.
SGJ_SLOTS_PER_EDGE = 4
# Coupling bitmap: every (row, column) pair is evaluated and masked by its
# bit, the row's 64-bit word of 64 senders serving as the lane mask of one
# select: v_sub, v_mul, v_exp_f32 (2 slots), v_fma, v_cndmask, v_fmac.
BITMAP_SLOTS_PER_PAIR = 7


def slots_of(n, path=None):
    """Issue slots of one network's step: its compartment updates plus its
    pair or edge work in the form the path evaluates it."""
    s = CELL_SLOTS * n.n
    if n.conn == "uniform":
        s += UNIFORM_SLOTS_PER_PAIR * n.n * n.n
    elif n.conn == "csr" and path == "csr_bitmap":
        s += BITMAP_SLOTS_PER_PAIR * n.n * n.n
    elif n.conn in ("csr", "dense"):
        s += (SGJ_SLOTS_PER_EDGE if n.gap == "sgj" else CSR_SLOTS_PER_EDGE) * n.pairs_per_step()
    return s


def step_kernel_name(info, nets):
    """The kernel(s) one step launches, from the context's launch groups and
    the variant the runtime picks for them: 1 when no network has gap
    junctions, 2 when none has per-edge weights or per-cell parameters,
    else 0."""
    if info["step_mode"] == 3:
        return "infoli::k_persist"
    if all(n.conn == "none" and n.cell_params is None for n in nets):
        var = 1
    elif all(n.w_csr is None and n.cell_params is None for n in nets):
        var = 2
    else:
        var = 0
    wide, total = info["n_tiles_wide"], info["n_tiles"]
    wblock = info.get("wide_threads", 1024)
    narrow = f"infoli::k_step<256, {var}>"
    if wide == 0:
        return narrow
    if wide == total:
        return f"infoli::k_step<{wblock}, {2 if var == 2 else 0}>"
    return f"{narrow} + infoli::k_step<{wblock}, {2 if var == 2 else 0}> (concurrent graph branches)"


def roofline(nets, launch_s, kernel="infoli::k_step<256, 2>", paths=None):
    """The roofline of one step launch. `paths`: the library's gap path per
    network (bytes and pair work are counted in the form it streams and
    evaluates); None takes the CSR gather format."""
    paths = paths if paths is not None else [None] * len(nets)
    kinds = {n.conn for n in nets}
    if len(kinds) > 1:
        # mixed batch: issue slots against the lane-slot peak; and the
        # composite bound, per network the larger of its bytes at the HBM
        # peak and its issue slots at the lane-slot peak, summed
        slots = sum(slots_of(n, p) for n, p in zip(nets, paths))
        achieved = slots / launch_s / 1e12
        peak = LANE_SLOTS_PER_S / 1e12
        t_roof = sum(max(algorithmic_bytes([n], [p]) / (HBM_PEAK_GBS * 1e9), slots_of(n, p) / LANE_SLOTS_PER_S)
                     for n, p in zip(nets, paths))
        return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "T lane-slots/s",
                "frac": achieved / peak, "traffic": None, "kernel": kernel,
                "slots_per_launch": slots, "composite_roofline_us": t_roof * 1e6,
                "composite_frac": t_roof / launch_s}
    if all(n.conn == "uniform" and n.gap == "rgj" for n in nets):
        pairs = sum(n.n * n.n for n in nets)       # the kernel evaluates the diagonal too
        achieved = pairs / launch_s / 1e9
        peak = LANE_SLOTS_PER_S / UNIFORM_SLOTS_PER_PAIR / 1e9
        # the exp-shared minimum: f(dV) = f(-dV), so one exp serves both directions
        peak_shared = LANE_SLOTS_PER_S / (UNIFORM_SLOTS_PER_PAIR - EXP_SLOTS / 2) / 1e9
        return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Gpair/s",
                "frac": achieved / peak, "traffic": None, "kernel": kernel,
                "slots_per_pair": UNIFORM_SLOTS_PER_PAIR, "pairs_per_launch": pairs,
                "frac_vs_exp_shared_minimum": achieved / peak_shared}
    abytes = algorithmic_bytes(nets, paths)
    if all(n.conn == "csr" for n in nets):
        # the larger of the two bounds: bytes at the HBM peak or issue slots
        # at the lane-slot peak (a network on the coupling bitmap streams few
        # bytes and evaluates every pair)
        slots = sum(slots_of(n, p) for n, p in zip(nets, paths))
        t_hbm = abytes / (HBM_PEAK_GBS * 1e9)
        t_alu = slots / LANE_SLOTS_PER_S
        extra = {"algorithmic_bytes_per_launch": abytes, "slots_per_launch": slots,
                 "hbm_frac": t_hbm / launch_s, "alu_frac": t_alu / launch_s,
                 "gap_paths": sorted(set(p or "csr_gather" for p in paths))}
        if t_alu > t_hbm:
            achieved = slots / launch_s / 1e12
            peak = LANE_SLOTS_PER_S / 1e12
            return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "T lane-slots/s",
                    "frac": achieved / peak, "traffic": None, "kernel": kernel, **extra}
        achieved = abytes / launch_s / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel, **extra}
    achieved = abytes / launch_s / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
           "algorithmic_bytes_per_launch": abytes}
    if all(n.conn == "none" or (n.conn == "uniform" and n.gap == "sgj") for n in nets):
        # issue-slot use of the compartment update's own arithmetic
        cells = sum(n.n for n in nets)
        out["alu_frac"] = CELL_SLOTS * cells / launch_s / LANE_SLOTS_PER_S
        out["alu_slots_per_cell_step"] = CELL_SLOTS
    return out


def cpu_baseline(nets, budget_s=15.0):
    """The fp32 oracle on the host cores, a bounded number of steps of the
    same networks (timed per network, summed)."""
    from oracle import Oracle, max_threads
    o = Oracle("f32")
    x0s = [o.initial_state(n) for n in nets]
    t0 = time.perf_counter()
    for n, x in zip(nets, x0s):
        o.run(n, 2, x0=x)
    probe = max(time.perf_counter() - t0, 1e-4) / 2.0
    steps = int(max(2, min(5000, budget_s / probe)))
    t0 = time.perf_counter()
    for n, x in zip(nets, x0s):
        o.run(n, steps, x0=x)
    dt = time.perf_counter() - t0
    cells = sum(n.n for n in nets)
    cores = max_threads()           # before the one-thread leg changes it
    # the same on one thread, within a third of the budget (skipped when one
    # step alone would take longer)
    est1 = dt / steps * cores
    single, steps1 = None, 0
    if est1 <= budget_s / 3.0:
        steps1 = int(max(1, min(steps, (budget_s / 3.0) / est1)))
        t0 = time.perf_counter()
        for n, x in zip(nets, x0s):
            o.run(n, steps1, x0=x, threads=1)
        single = cells * steps1 / (time.perf_counter() - t0)
    return {"value": cells * steps / dt, "unit": "cell-steps/s", "cores": cores,
            "kind": "oracle", "single_thread_value": single,
            "sample": f"{steps} steps ({steps1} on one thread) of the same {len(nets)} network(s) ({cells} cells) "
                      "from the initial state, fp32 oracle, OpenMP over cells"}


def run_validation(nets, desc, steps, warmup, args, torch, infoli):
    """The long run with per-step output streaming (output ring, copies of
    each 1,000-step chunk queued on the library's copy stream into pinned
    host memory) against the same run without it."""
    net = nets[0]
    x0 = infoli.initial_state(net)
    chunk, ring = 1000, 2000
    host = torch.zeros((steps, net.n), dtype=torch.float32, pin_memory=True)
    hv = host.numpy()
    times = {}
    for streamed in (False, True):
        opt = {"output_ring_steps": ring} if streamed else {}
        sim = infoli.Simulator(net, init_states=[x0], step_mode=args.mode, **opt)
        mode = sim.info()["step_mode"]
        sim.step(warmup)
        sim.sync()
        sim.write_state(0, x0, 0)
        sim.clear_spikes()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s0 in range(0, steps, chunk):
            sim.step(chunk)
            if streamed:
                view = hv[s0:s0 + chunk]
                sim.output_copy_async(s0, chunk, view.ctypes.data, view.size)
        if streamed:
            sim.output_wait()
        sim.sync()
        times[streamed] = time.perf_counter() - t0
        counts, _ = sim.read_spikes(0)
        last = sim.read_state(0)
        sim.close()
    va = hv
    crossings = ((va[:-1] < 0.0) & (va[1:] >= 0.0)).sum(axis=0) + ((x0[I.IDX_VA] < 0.0) & (va[0] >= 0.0))
    out = {
        "metric": "cell-steps/sec (plain InfOli step) with per-step output streamed to the host",
        "value": net.n * steps / times[True],
        "unit": "cell-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": times[True] * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"valid120k: {desc}", "cells": net.n, "step_mode": mode,
                   "chunk_steps": chunk, "ring_steps": ring},
        "us_per_step_streamed": times[True] * 1e6 / steps,
        "us_per_step_not_streamed": times[False] * 1e6 / steps,
        "streaming_overhead": times[True] / times[False] - 1.0,
        "real_time_factor": (steps * net.dt * 1e-3) / times[True],
        "output_bytes_streamed": int(steps * net.n * 4),
        "spikes_counted_by_library": int(counts.sum()),
        "spikes_in_streamed_output": int(crossings.sum()),
        "streamed_last_step_equals_state": bool(np.array_equal(va[-1], last[I.IDX_VA])),
    }
    print(json.dumps(out), flush=True)


def run_surrogate(nets, desc, steps, warmup, args, torch, infoli):
    """Plain run vs trained surrogate on the same network and initial state."""
    net = nets[0]
    x0 = infoli.initial_state(net)
    V = [I.IDX_VD, I.IDX_VS, I.IDX_VA]
    macro = steps // 4
    samples = 25
    every = macro // samples
    # plain method
    plain = infoli.Simulator(net, init_states=[x0], step_mode="graph", graph_chunk=100)
    info = plain.info()
    paths = [plain.gap_path(0)[0]]
    ref, t_plain = [], 0.0
    for _ in range(samples):
        plain.step(4 * every)
        plain.sync()
        t_plain += plain.last_step_ms()
        ref.append(plain.read_state(0)[V])
    ca, ta = plain.read_spikes(0)
    plain.close()
    # training
    sim = infoli.Simulator(net, init_states=[x0], step_mode="graph", graph_chunk=100)
    t0 = time.perf_counter()
    rep, hist = sim.surrogate_train(I.mlp_init_params(5000))
    train_wall = time.perf_counter() - t0
    params, norm = sim.surrogate_get()
    sim.close()

    def surrogate_run(**drift):
        s = infoli.Simulator(net, init_states=[x0], step_mode="graph", graph_chunk=100)
        s.surrogate_set(params, norm)
        sq, n, ms, checked, flagged, plain_cells = 0.0, 0, 0.0, 0, 0, 0
        for k in range(samples):
            r = s.step_surrogate(every, **drift)
            ms += r["ms"]
            checked += r["checked"]
            flagged += r["flagged"]
            plain_cells += r["plain_cell_macro_steps"]
            d = (s.read_state(0)[V] - ref[k]).astype(np.float64)
            sq += float((d * d).sum())
            n += d.size
        cb, tb = s.read_spikes(0)
        s.close()
        worst = 0.0
        for i in np.nonzero((ca > 0) & (cb > 0))[0]:
            m = min(ca[i], cb[i], ta.shape[1])
            worst = max(worst, float(np.max(np.abs(np.sort(ta[i, :m]) - np.sort(tb[i, :m])))))
        return {"ms": ms, "rmse_mv": float(np.sqrt(sq / n)), "spikes": int(cb.sum()),
                "spike_count_max_diff": int(np.max(np.abs(ca.astype(np.int64) - cb))),
                "spike_time_err_ms": worst, "checked": checked, "flagged": flagged,
                "plain_cell_macro_steps": plain_cells}

    surr = surrogate_run()
    hold = surrogate_run(mode="plain_hold")
    nofb = surrogate_run(sample_every=0, v_max=1e30, z_max=0.0)
    cells = net.n
    total_steps = 4 * every * samples
    out = {
        "metric": "surrogate vs plain speedup at voltage RMSE <= 1 mV (cell-steps/s of the surrogate path)",
        "value": cells * total_steps / (surr["ms"] * 1e-3),
        "unit": "cell-steps/s",
        "n_gpus": 1, "steps": total_steps, "warmup": 0,
        "ms_per_step": surr["ms"] / total_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": f"surr65k: {desc}", "cells": cells, "gap_pairs_per_step": net.pairs_per_step(),
                   "tiles": info["n_tiles"], "tiles_wide": info["n_tiles_wide"], "wide_threads": info["wide_threads"],
                   "csr_bitmap_networks": info["n_bitmap"], "csr_blocked_networks": info["n_blocked"],
                   "lanes_per_row": info["lanes_per_row"]},
        "plain_cell_steps_per_s": cells * total_steps / (t_plain * 1e-3),
        "plain_ms_per_step": t_plain / total_steps,
        "speedup": t_plain / surr["ms"],
        "rmse_mv": surr["rmse_mv"], "spike_time_err_ms": surr["spike_time_err_ms"],
        "spikes_plain": int(ca.sum()), "spikes_surrogate": surr["spikes"],
        "drift": {k: surr[k] for k in ("checked", "flagged", "plain_cell_macro_steps")},
        "ablation_held_gap_no_mlp": {"speedup": t_plain / hold["ms"], "rmse_mv": hold["rmse_mv"]},
        "ablation_mlp_no_fallback": {"speedup": t_plain / nofb["ms"], "rmse_mv": nofb["rmse_mv"],
                                     "spike_time_err_ms": nofb["spike_time_err_ms"]},
        "training": {**rep, "wall_s": train_wall},
        "roofline": roofline(nets, t_plain * 1e-3 / total_steps, step_kernel_name(info, nets), paths),
    }
    out["roofline"]["traffic"] = measured_traffic(args.workload)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nets, args.cpu_budget)
    print(json.dumps(out), flush=True)


def copy_probe(mb, torch):
    """A plain device copy of known size: HBM counter calibration for
    rocprofv3, and the copy bandwidth this GPU reaches (HIP events)."""
    n = int(mb * 1024 * 1024 // 4)
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / 3
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 5,
                      "copy_GBps_read_plus_write": 8 * n / s / 1e9}))


# Table 3 of the paper (largest network run in real time, 50 us of simulated
# time per step, on its three platforms), quoted as context.
PAPER_TABLE3 = {
    "hardware": {"DFE": "Maxeler Maia DFE (Altera Stratix V 5SGSD8)", "Xeon Phi": "Intel Xeon Phi 5110P",
                 "GPU": "NVIDIA Titan X (Maxwell)"},
    "RGJ 100%": {"DFE": 310}, "RGJ 75%": {"DFE": 310}, "RGJ 50%": {"DFE": 310}, "RGJ 25%": {"DFE": 310},
    "SGJ 100%": {"DFE": 400}, "SGJ 75%": {"DFE": 400}, "SGJ 50%": {"DFE": 400, "GPU": 96},
    "SGJ 25%": {"DFE": 400, "GPU": 96}, "NGJ": {"DFE": 7680, "Xeon Phi": 96, "GPU": 500},
}


def rt_network(case, n):
    """One network of the real-time sweep: 100 % density is all-to-all,
    lower densities symmetric ER graphs as CSR, NGJ uncoupled; conductance
    0.04 * 96 / (density * N) (the summed coupling of the 96-cell network),
    jitter, bias N(0, 0.5)."""
    kind, dens = case.split()[0].lower(), case.split()[-1]
    jit, bias = I.voltage_jitter(n, 2000), I.input_bias(n, 3000)
    if kind == "ngj":
        return I.Network(n=n, conn="none", jitter=jit, bias=bias)
    d = float(dens.rstrip("%")) / 100.0
    g = 0.04 * 96.0 / (d * n)
    if d >= 1.0:
        return I.Network(n=n, conn="uniform", g=g, jitter=jit, bias=bias, gap=kind)
    rp, col = I.erdos_renyi_csr(n, d, 1000)
    return I.Network(n=n, conn="csr", g=g, row_ptr=rp, col=col, jitter=jit, bias=bias, gap=kind)


def rt_sweep(args, torch, infoli):
    """Largest network per use case and density whose steps take at most
    the real-time budget (Section 2.2: 50 us of simulated time per step):
    sizes on a grid of ratio sqrt(2) (multiples of 32) from 96 up to the
    first size over budget; each size timed over 300 steps after 50 warm-up
    steps in the library's automatic launch mode."""
    budget = args.rt_budget_us
    cases = ["RGJ 100%", "RGJ 75%", "RGJ 50%", "RGJ 25%", "SGJ 100%", "SGJ 75%", "SGJ 50%", "SGJ 25%", "NGJ"]
    max_edges = 2.6e8
    out = []
    for case in cases:
        points, best, first_over = [], None, None
        k = 0
        while True:
            n = int(round(96 * 2 ** (k / 2) / 32.0)) * 32
            k += 1
            dens = 1.0 if case == "NGJ" else float(case.split()[-1].rstrip("%")) / 100.0
            if case != "NGJ" and 0 < dens < 1.0 and dens * n * n > max_edges:
                break
            if n > (1 << 24):
                break
            net = rt_network(case, n)
            sim = infoli.Simulator([net], init_states=[infoli.initial_state(net)], step_mode="auto")
            sim.step(50)
            sim.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(300)
            torch.cuda.synchronize()
            us = (time.perf_counter() - t0) / 300 * 1e6
            mode = sim.info()["step_mode"]
            sim.close()
            points.append([n, round(us, 2)])
            print(f"rt {case} n={n} {us:.2f} us/step (mode {mode})", file=sys.stderr, flush=True)
            if us <= budget:
                best = [n, round(us, 2)]
            else:
                first_over = [n, round(us, 2)]
                break
        out.append({"case": case, "max_cells": best[0] if best else 0,
                    "us_per_step_at_max": best[1] if best else None,
                    "first_over_budget": first_over, "points": points})
    print(json.dumps({"rt_sweep": {"budget_us": budget, "cases": out,
                                   "paper_table3_context": PAPER_TABLE3}}), flush=True)


# Table 4's scenario (Section 3.3): per network size a batch of five
# realistic-gap experiments at 100, 75, 50, 25 and 0 % density, 40 s of
# brain time (800,000 steps) each. The average time per step that BrainFrame
# (the best fabric per experiment) reaches there, derived from Table 4's
# savings, is quoted as context.
PAPER_TABLE4_BRAINFRAME_US_PER_STEP = {384: 58.0, 960: 303.0, 5760: 2210.0, 7680: 13300.0}


def paper_batches(args, torch, infoli):
    """Table 4's batches on one MI355X: every experiment alone (one after
    the other, as on one accelerator) and all five in one batched context
    (one launch per step), each timed over 500 steps after 50 warm-up
    steps; batch time = steps per experiment x the per-step times."""
    steps_per_exp = 800000
    out = []
    for n in (384, 960, 5760, 7680):
        nets = [rt_network(c, n) for c in ("RGJ 100%", "RGJ 75%", "RGJ 50%", "RGJ 25%")]
        nets.append(I.Network(n=n, conn="none", jitter=I.voltage_jitter(n, 2000), bias=I.input_bias(n, 3000)))

        def per_step(group):
            sim = infoli.Simulator(group, init_states=[infoli.initial_state(x) for x in group])
            sim.step(50)
            sim.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(500)
            torch.cuda.synchronize()
            us = (time.perf_counter() - t0) / 500 * 1e6
            sim.close()
            return us

        alone = [per_step([x]) for x in nets]
        together = per_step(nets)
        seq_s = sum(alone) * 1e-6 * steps_per_exp
        bat_s = together * 1e-6 * steps_per_exp
        paper_s = PAPER_TABLE4_BRAINFRAME_US_PER_STEP[n] * 1e-6 * 5 * steps_per_exp
        row = {"cells": n, "us_per_step_alone": [round(u, 2) for u in alone],
               "us_per_step_five_batched": round(together, 2),
               "batch_seconds_one_after_another": round(seq_s, 2), "batch_seconds_batched": round(bat_s, 2),
               "paper_brainframe_batch_seconds": round(paper_s, 1),
               "speedup_vs_brainframe_batched": round(paper_s / bat_s, 1)}
        print(f"paper batch n={n}: alone {row['us_per_step_alone']} us, batched {together:.2f} us per step",
              file=sys.stderr, flush=True)
        out.append(row)
    print(json.dumps({"paper_batches": {
        "scenario": "Table 4: five RGJ experiments (100/75/50/25/0 % density) of 800,000 steps per network size",
        "densities": ["100% (all-to-all)", "75% (ER CSR)", "50%", "25%", "0% (no gap junctions)"],
        "paper_context": "BrainFrame's average time per step (derived from Table 4's savings) on its three "
                         "fabrics (Maxeler Maia DFE, Xeon Phi 5110P, Titan X), the best fabric per experiment",
        "sizes": out}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="csr4096", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="auto", choices=["graph", "launch", "auto", "persistent"])
    ap.add_argument("--graph-chunk", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--rt-sweep", action="store_true",
                    help="only run the real-time size sweep (largest network per use case within the budget)")
    ap.add_argument("--rt-budget-us", type=float, default=50.0)
    ap.add_argument("--paper-batches", action="store_true",
                    help="only run Table 4's experiment batches (per size, five densities)")
    ap.add_argument("--copy-probe-mb", type=float, default=0.0,
                    help="only run a device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the per-step Vd exchange across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    steps = args.steps if args.steps is not None else WORKLOADS[args.workload]["steps"]
    warmup = args.warmup if args.warmup is not None else WORKLOADS[args.workload]["warmup"]

    import torch
    from paper_1612_01501_amd import infoli
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mb > 0:
        copy_probe(args.copy_probe_mb, torch)
        return
    if args.rt_sweep:
        rt_sweep(args, torch, infoli)
        return
    if args.paper_batches:
        paper_batches(args, torch, infoli)
        return
    nets, desc = build_workload(args.workload)
    if args.workload == "surr65k":
        run_surrogate(nets, desc, steps, warmup, args, torch, infoli)
        return
    if args.workload == "valid120k":
        run_validation(nets, desc, steps, warmup, args, torch, infoli)
        return
    x0s = [infoli.initial_state(n) for n in nets]
    stream = torch.cuda.current_stream().cuda_stream
    sim = infoli.Simulator(nets, init_states=x0s, stream=stream, step_mode=args.mode,
                           graph_chunk=args.graph_chunk)
    info = sim.info()
    paths = [sim.gap_path(k)[0] for k in range(len(nets))]
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    dev_ms = sim.last_step_ms()
    sim.close()

    cells = sum(n.n for n in nets)
    pairs = sum(n.pairs_per_step() for n in nets)
    cell_steps_s = cells * steps / wall
    launch_s = dev_ms * 1e-3 / steps        # one step kernel launch per step
    out = {
        "metric": "cell-steps/sec (plain InfOli step, gap junctions + compartments)",
        "value": cell_steps_s,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "cells": cells,
                   "gap_pairs_per_step": pairs, "step_mode": args.mode,
                   "tiles": info["n_tiles"], "tiles_wide": info["n_tiles_wide"], "wide_threads": info["wide_threads"],
                   "csr_bitmap_networks": info["n_bitmap"], "csr_blocked_networks": info["n_blocked"],
                   "lanes_per_row": info["lanes_per_row"]},
        "gap_pairs_per_s": pairs * steps / wall,
        "device_ms_per_step": dev_ms / steps,
        "roofline": roofline(nets, launch_s, step_kernel_name(info, nets), paths),
    }
    out["roofline"]["traffic"] = measured_traffic(args.workload)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nets, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
