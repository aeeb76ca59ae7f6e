#!/usr/bin/env python3
"""Throughput of the InfOli step on one MI355X.

A "step" advances every network of the workload by one synchronous time step
(dt = 0.05 ms): gap-junction currents plus the three-compartment update of
every cell, all in the library's HIP kernels. Inputs are synthetic (seeded),
shaped like the paper's networks, and resident in device memory before the
timed region starts.

Workloads (--workload):
  c4       the default: 65,536 cells, symmetric ER graph of mean degree 1,000
           (CSR, 65.5 M edges, g = 3.84e-3), bias N(0, 0.5), pulse, jitter;
           the plain step timed over --steps steps (every one a replay of a
           HIP graph captured at init), then the trained MLP surrogate
           against the plain method over 10,000 dt (2,500 macro steps of
           4 dt, drift check 1/64 cells, theta 0.5 mV) with the two ablations
           (held gap without MLP; MLP without fallback), and the same under
           the paper's 25 ms validation pulse where cells fire
  csr4096  three 4,096-cell symmetric Erdos-Renyi CSR networks at 1 %, 10 %
           and 50 % density (g = 0.04, bias N(0, 0.5), 6 uA/cm^2 pulse at
           20-25 ms), stepped together, 20,000 steps
  uni96    96 cells all-to-all (g = 0.04), 2,000 steps
  uni16k   16,384 cells all-to-all (g = 0.04*96/N), 4,000 steps
  csr65k   the c4 network stepped by the plain method only, 2,000 steps
  ngj16m   2^24 uncoupled cells: the compartment update alone, 1.95 GB of
           state per step (beyond the 256 MB cache), 200 steps
  valid120k the paper's validation run: 96 cells, 25 ms pulse, 120,000 steps
           (6 s) with every step's axon voltages streamed to the host
  sgj65k   the csr65k network with simplified gap junctions (w * dV), 2,000
           steps
  sgj16k   the uni16k network with simplified gap junctions (the closed
           form g (N Vd_i - sum Vd)), 4,000 steps
  sgj1m    2^20 cells all-to-all with simplified gap junctions, the sum of
           all voltages taken once per step, 2,000 steps (no CPU baseline:
           the oracle evaluates all 1.1e12 pairs of a step)
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


def code_of(text):
    """C/C++ source without its comments, whitespace runs collapsed: what the
    compiler sees, so that an edit of a comment leaves the hash alone."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":                              # a string or character literal, kept
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash():
    """Hash of the kernel sources' code (comments and layout excluded)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(code_of(fh.read()).encode())
    return h.hexdigest()[:16]


def traffic_key(workload, kernel, paths, info):
    """What the counters must have been taken on to count for this run: the
    workload, the step kernel(s), the gap paths and the wide workgroup size."""
    return "|".join([workload, kernel, ",".join(sorted(set(p or "csr_gather" for p in paths))),
                     f"wide{info.get('wide_threads', 0)}"])


def measured_traffic(key):
    """Measured HBM bytes per launch for exactly this configuration (see
    traffic_key), or None when no counters were taken for it or the kernel
    sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            entry = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not entry or entry.get("kernel_sources_sha256") != kernel_source_hash():
        return None
    return entry["bytes_per_launch"]


def _counter_rows(run_dir):
    """Per-dispatch values of one rocprofv3 --pmc run (its *counter_collection.csv
    under run_dir): list of (dispatch id, kernel name, counter, value)."""
    import csv
    import glob
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit(f"{run_dir}: expected one counter_collection.csv, found {len(files)}")
    with open(files[0]) as fh:
        return [(int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]))
                for r in csv.DictReader(fh)]


def _per_dispatch(rows, counter, name_part, last):
    """The counter summed per dispatch over the `last` dispatches of the
    kernel whose name contains name_part (the timed ones come last)."""
    per = {}
    for d, k, c, v in rows:
        if c == counter and name_part in k:
            per[d] = per.get(d, 0.0) + v
    ids = sorted(per)
    if last and len(ids) < last:
        raise SystemExit(f"only {len(ids)} dispatches of {name_part!r} with {counter}, expected >= {last}")
    ids = ids[-last:] if last else ids
    return [per[d] for d in ids]


def ingest_traffic(run_root):
    """Turn the four counter runs under run_root (copy_fetch, copy_write: the
    plain copy of --copy-probe-mb; fetch, write: the benchmark, whose JSON
    lines are fetch.json and write.json) into the HBM bytes per step-kernel
    launch, stored in the traffic file under the benchmark's traffic key."""
    with open(os.path.join(run_root, "copy.json")) as fh:
        copy = json.loads(fh.read().strip().splitlines()[-1])
    runs = {}
    for k in ("fetch", "write"):
        with open(os.path.join(run_root, f"{k}.json")) as fh:
            runs[k] = json.loads(fh.read().strip().splitlines()[-1])
    key = runs["fetch"]["roofline"]["traffic_key"]
    if runs["write"]["roofline"]["traffic_key"] != key:
        raise SystemExit("the FETCH_SIZE and WRITE_SIZE runs ran different configurations")
    r = runs["fetch"]
    n = r["steps"] + r["warmup"]
    # a step of two kernels ("A + B") adds both kernels' bytes
    parts = [p.strip().replace("infoli::", "")
             for p in r["roofline"]["kernel"].split("(concurrent")[0].split(" + ")]
    cf = _per_dispatch(_counter_rows(os.path.join(run_root, "copy_fetch")), "FETCH_SIZE", "", 0)
    cw = _per_dispatch(_counter_rows(os.path.join(run_root, "copy_write")), "WRITE_SIZE", "", 0)
    copy_kib = copy["copy_probe_bytes_read"] / 1024.0
    # the copy is the largest dispatch of its run
    fetch_factor = copy_kib / max(cf)
    write_factor = copy_kib / max(cw)
    frows = _counter_rows(os.path.join(run_root, "fetch"))
    wrows = _counter_rows(os.path.join(run_root, "write"))
    fk = wk = 0.0
    for kname in parts:
        f = _per_dispatch(frows, "FETCH_SIZE", kname, n)
        w = _per_dispatch(wrows, "WRITE_SIZE", kname, n)
        fk, wk = fk + float(np.mean(f)), wk + float(np.mean(w))
    entry = {"kernel": r["roofline"]["kernel"], "dispatches": [len(f), len(w)],
             "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
             "fetch_factor": round(fetch_factor, 4), "write_factor": round(write_factor, 4),
             "bytes_per_launch": int(round(1024.0 * (fk * fetch_factor + wk * write_factor))),
             "algorithmic_bytes_per_launch": r["roofline"].get("algorithmic_bytes_per_launch"),
             "kernel_sources_sha256": kernel_source_hash()}
    try:
        with open(TRAFFIC_FILE) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        table = {}
    table[key] = entry
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps({key: entry}))


def tuned_config(info, sim, nets):
    """What the library runs for these networks, as chosen at init."""
    return {"tiles": info["n_tiles"], "tiles_wide": info["n_tiles_wide"], "wide_threads": info["wide_threads"],
            "csr_bitmap_networks": info["n_bitmap"], "csr_blocked_networks": info["n_blocked"],
            "lanes_per_row": info["lanes_per_row"], "tile_rows": info["tile_rows"],
            "gap_paths": sorted(set(sim.gap_path(k)[0] for k in range(len(nets)))),
            "step_kernel": step_kernel_name(info, nets, [sim.gap_path(k)[0] for k in range(len(nets))]),
            "tuned_networks": info["tuned"], "tune_cached_networks": info["tune_cached"],
            "csr_stream_networks": info["n_stream"], "tune_mode": info["tune_mode"],
            "stream_round": info["stream_round"], "unordered_pair_networks": info["n_sym"]}


WORKLOADS = {
    "c4": dict(steps=2000, warmup=100),
    "csr4096": dict(steps=20000, warmup=1000),
    "uni96": dict(steps=2000, warmup=200),
    "uni16k": dict(steps=4000, warmup=100),
    "batch256": dict(steps=10000, warmup=200),
    "csr65k": dict(steps=2000, warmup=100),
    "ngj16m": dict(steps=200, warmup=10),
    "valid120k": dict(steps=120000, warmup=1000),
    "sgj65k": dict(steps=2000, warmup=100),
    "sgj16k": dict(steps=4000, warmup=200),
    "sgj1m": dict(steps=2000, warmup=100),
}
# workloads whose oracle step is beyond a bounded CPU sample
NO_CPU_BASELINE = {"sgj1m": "the oracle evaluates every pair by its definition, 1.1e12 per step"}


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
    elif name == "c4":
        nets = [I.config4()]
        desc = ("65,536 cells, symmetric ER gap graph of mean degree 1,000 (CSR, 65.5 M edges), g=3.84e-3 mS/cm^2, "
                "bias N(0,0.5), 6 uA/cm^2 pulse steps [400,500), +-1 mV jitter, FP32, dt=0.05 ms; plain step "
                "throughput, then the MLP surrogate (16-128-128-16, BF16 on MFMA, 4 dt per macro step, drift "
                "check 1/64 cells) against the plain method over 10,000 dt")
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
    elif name == "sgj1m":
        nets = [I.config2(n=1 << 20)]
        nets[0].gap = "sgj"
        desc = ("1,048,576 cells all-to-all, simplified gap junctions w*dV (closed form g*(N*Vd_i - sum Vd), "
                "the sum taken once per step), g=0.04*96/N mS/cm^2, +-1 mV jitter, no input, FP32, dt=0.05 ms")
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


# Issue slots: one slot is one wave64 lane of a full-rate FP32 VALU
# operation (FMA class). The lane-slot peak is MI355X's FP32 vector peak,
# 157.3 TFLOP/s = 78.6 T FMA/s = 256 CUs x 128 lanes x 2.4 GHz; plain
# (unpacked) v_fma_f32 reaches it (a register-only loop: 6.27e13 FMA/s at the
# clock under load). The transcendentals v_exp_f32 and v_rcp_f32 cost
# EXP_SLOTS = 3.3 slots each (the same loop: 1.89e13 exp/s, 3.3x fewer), and
# do not overlap with the FMA-class operations around them (the pair term's
# sub / mul / exp / fma mix runs at 7.7 slots per pair, not max(3, 3.3)).
LANE_SLOTS_PER_S = 256 * 128 * 2.4e9
EXP_SLOTS = 3.3
# Uniform all-to-all kernel: per directed pair one v_sub, one v_mul, one
# v_exp_f32 and one v_fma (w = g factored out, the linear 0.2*dV part in
# closed form).
UNIFORM_SLOTS_PER_PAIR = 3 + EXP_SLOTS
# The same networks with each unordered pair once (k_pairs_sym): per pair
# one v_sub, v_mul, v_exp_f32 and two v_fma (the row's sum and the column's).
SYM_SLOTS_PER_PAIR = 4 + EXP_SLOTS
# Compartment update per cell-step: 278 VALU instructions in its compiled
# form, of which 39 transcendental (21 v_exp_f32, 18 v_rcp_f32).
CELL_SLOTS = 278 - 39 + 39 * EXP_SLOTS


def algorithmic_bytes(nets, paths=None):
    """Bytes one step launch must move at minimum, in the format each network
    is streamed in (`paths`: the library's gap path per network; None takes
    the CSR gather format): per cell 14 state floats in and out plus the bias
    (116 B); per CSR edge its column (uint16 when every CSR network has
    <= 65,536 cells, else int32) plus its fp32 weight when the network has
    per-edge weights, and per CSR row its row pointer (8 B); for a network on
    the coupling bitmap instead, one bit per (row, column) pair in rows of
    whole 32-bit words; for a network on the chunk stream, also one byte per
    eight edges (the row tag of each chunk; padding not counted). Gathered
    neighbour voltages are cache hits and not counted."""
    col_b = 2 if all(n.n <= 65536 for n in nets if n.conn == "csr") else 4
    b = 0
    for k, n in enumerate(nets):
        b += 116 * n.n
        if n.conn == "csr" and paths is not None and paths[k] == "csr_bitmap":
            b += 4 * n.n * ((n.n + 31) // 32)
        elif n.conn == "csr":
            nnz = int(n.row_ptr[-1])
            b += (col_b + (4 if n.w_csr is not None else 0)) * nnz + 8 * n.n
            if paths is not None and paths[k] == "csr_stream":
                b += nnz // 8        # the one-byte row tag of each chunk of eight columns
        elif n.conn == "dense":
            b += 4 * n.n * n.n
    return b


# CSR edge: v_sub, v_mul, v_mul, v_exp_f32, v_fma, v_add and two address
# operations for the 16-bit column gather.
CSR_SLOTS_PER_EDGE = 7 + EXP_SLOTS
# Simplified gap junctions, per CSR edge: v_sub, v_fma and the two address
# operations.
SGJ_SLOTS_PER_EDGE = 4
# Coupling bitmap: every (row, column) pair is evaluated and masked by its
# bit, the row's 64-bit word of 64 senders serving as the lane mask of one
# select: v_sub, v_mul, v_exp_f32, v_fma, v_cndmask, v_fmac.
BITMAP_SLOTS_PER_PAIR = 5 + EXP_SLOTS


def slots_of(n, path=None):
    """Issue slots of one network's step: its compartment updates plus its
    pair or edge work in the form the path evaluates it."""
    s = CELL_SLOTS * n.n
    if n.conn == "uniform" and path == "uniform_sym":
        own = (n.n + 63) // 64 * 64 * 64
        s += SYM_SLOTS_PER_PAIR * (n.n * n.n - own) / 2 + UNIFORM_SLOTS_PER_PAIR * own
    elif n.conn == "uniform":
        s += UNIFORM_SLOTS_PER_PAIR * n.n * n.n
    elif n.conn == "csr" and path == "csr_bitmap":
        s += BITMAP_SLOTS_PER_PAIR * n.n * n.n
    elif n.conn in ("csr", "dense"):
        s += (SGJ_SLOTS_PER_EDGE if n.gap == "sgj" else CSR_SLOTS_PER_EDGE) * n.pairs_per_step()
    return s


def step_kernel_name(info, nets, paths=None):
    """The kernel(s) one step launches, from the context's launch groups and
    the variant the runtime picks for them: 1 when no network has gap
    junctions, 3 when every network runs the chunk stream (the wide group
    only), 2 when none has per-edge weights or per-cell parameters, else 0."""
    if info["step_mode"] == 3:
        return "infoli::k_persist"
    if paths and any(p == "uniform_sym" for p in paths):
        rest = step_kernel_name(info, nets, [p if p != "uniform_sym" else "uniform" for p in paths])
        return "infoli::k_pairs_sym + " + rest
    if paths and any(p == "uniform_sum" for p in paths):
        rest = step_kernel_name(info, nets, [p if p != "uniform_sum" else "uniform" for p in paths])
        return "infoli::k_vsum + " + rest
    if paths and all(p == "csr_stream" for p in paths):
        return f"infoli::k_step<{info.get('wide_threads', 1024)}, 3>"
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
    if all(n.conn == "uniform" and n.gap == "rgj" for n in nets) and all(p == "uniform_sym" for p in paths):
        # each unordered pair once: issue slots of the pair kernel's work
        # (a block's own 64 x 64 pairs ordered, as it evaluates them) and of
        # the compartment updates, at the lane-slot peak
        slots = 0.0
        for n in nets:
            blocks = (n.n + 63) // 64
            own = blocks * 64 * 64
            slots += SYM_SLOTS_PER_PAIR * (n.n * n.n - own) / 2 + UNIFORM_SLOTS_PER_PAIR * own + CELL_SLOTS * n.n
        achieved = slots / launch_s / 1e12
        peak = LANE_SLOTS_PER_S / 1e12
        ordered = sum(n.n * n.n for n in nets) / launch_s
        return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "T lane-slots/s",
                "frac": achieved / peak, "traffic": None, "kernel": kernel, "slots_per_launch": slots,
                "slots_per_unordered_pair": SYM_SLOTS_PER_PAIR, "gap_paths": ["uniform_sym"],
                "ordered_pair_frac": ordered / (LANE_SLOTS_PER_S / UNIFORM_SLOTS_PER_PAIR)}
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


def graph_chunk_for(steps, cap=100):
    """The largest even number of steps <= cap that divides `steps` (so every
    timed step is a graph replay), else 2."""
    for c in range(min(cap, steps) - (min(cap, steps) % 2), 1, -2):
        if steps % c == 0:
            return c
    return 2


def match_spikes(ca, ta, cb, tb, cap):
    """Per cell, greedy nearest-time matching of the kept spike times of run b
    to those of run a (each used once). Returns (abs time differences of the
    matched pairs, spikes of a left unmatched, spikes of b left unmatched)."""
    diffs, un_a, un_b = [], 0, 0
    for i in np.nonzero((ca > 0) | (cb > 0))[0]:
        a = np.sort(ta[i, :min(int(ca[i]), cap)].astype(np.float64))
        b = list(np.sort(tb[i, :min(int(cb[i]), cap)].astype(np.float64)))
        for t in a:
            if not b:
                un_a += 1
                continue
            k = int(np.argmin([abs(t - u) for u in b]))
            diffs.append(abs(t - b.pop(k)))
        un_b += len(b)
        un_a += max(0, int(ca[i]) - cap)
        un_b += max(0, int(cb[i]) - cap)
    return np.array(diffs), un_a, un_b


def stability(nets):
    """dt * lambda_max / C_m of the gap coupling linearised at synchrony
    (d/d(dV) of dV*(0.8*exp(-dV^2/100) + 0.2) is 1 at dV = 0, so the coupling
    is the weighted graph Laplacian), bounded by Gershgorin's 2*max_i sum_j
    w_ij; explicit Euler is stable for values <= 2 (C_m = 1 uF/cm^2)."""
    vals = []
    for n in nets:
        if n.conn == "uniform":
            row = (n.n - 1) * n.g
        elif n.conn == "csr":
            deg = np.diff(np.asarray(n.row_ptr))
            row = float(np.max(deg)) * n.g if n.w_csr is None else float(
                np.max(np.add.reduceat(np.asarray(n.w_csr, np.float64), np.asarray(n.row_ptr[:-1])))) if len(n.col) else 0.0
        elif n.conn == "dense":
            row = float(np.max(np.asarray(n.w_dense, np.float64).sum(axis=1)))
        else:
            row = 0.0
        vals.append(n.dt * 2.0 * row)
    vals = np.array(vals)
    return {"dt_lambda_max_gershgorin": float(vals.max()), "networks": len(vals),
            "networks_above_2": int((vals > 2.0).sum()), "euler_stable": bool((vals <= 2.0).all())}


def time_plain(sim, steps, warmup, torch):
    """Wall time of exactly `steps` steps between device synchronisations
    after `warmup` untimed ones, and the device time of the same call (HIP
    events on the context's stream)."""
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    return wall, sim.last_step_ms()


SURR_DT = 10000          # the surrogate comparison's length in dt, whatever --steps says
SURR_SAMPLES = 25


def surrogate_leg(net, x0, sim, torch, infoli, log, load=None, save=None):
    """Plain method against the trained MLP surrogate on the same network
    and initial state for SURR_DT time steps (SURR_DT / 4 macro steps), with
    the two ablations (held gap without MLP; MLP without fallback). `sim` is
    the plain context, rewound to x0 at step 0 for each run. `load`: take
    the weights and normalisation from this .npz instead of training;
    `save`: write the trained ones there."""
    V = [I.IDX_VD, I.IDX_VS, I.IDX_VA]
    every = SURR_DT // 4 // SURR_SAMPLES            # macro steps per sample
    cap = sim.spike_cap
    sim.write_state(0, x0, 0)
    sim.clear_spikes()
    ref, t_plain = [], 0.0
    for _ in range(SURR_SAMPLES):
        sim.step(4 * every)
        sim.sync()
        t_plain += sim.last_step_ms()
        ref.append(sim.read_state(0)[V])
    ca, ta = sim.read_spikes(0)
    log("surrogate leg: plain reference done")
    t0 = time.perf_counter()
    if load:
        with np.load(load) as z:
            sim.surrogate_set(z["params"], z["norm"])
        rep = {"loaded_from": load}
    else:
        rep, _ = sim.surrogate_train(I.mlp_init_params(5000))
        if save:
            params, norm = sim.surrogate_get()
            np.savez(save, params=params, norm=norm)
    train_wall = time.perf_counter() - t0
    log(f"surrogate leg: {'loaded' if load else 'trained'} ({train_wall:.1f} s)")

    def run(**drift):
        sim.write_state(0, x0, 0)
        sim.clear_spikes()
        sq, n, ms, checked, flagged, plain_cells, guarded = 0.0, 0, 0.0, 0, 0, 0, 0
        for k in range(SURR_SAMPLES):
            r = sim.step_surrogate(every, **drift)
            ms += r["ms"]
            checked += r["checked"]
            flagged += r["flagged"]
            plain_cells += r["plain_cell_macro_steps"]
            guarded += r["guarded"]
            d = (sim.read_state(0)[V] - ref[k]).astype(np.float64)
            sq += float((d * d).sum())
            n += d.size
        cb, tb = sim.read_spikes(0)
        diffs, un_a, un_b = match_spikes(ca, ta, cb, tb, cap)
        return {"ms": ms, "rmse_mv": float(np.sqrt(sq / n)), "spikes": int(cb.sum()),
                "spike_time_err_ms_max": float(diffs.max()) if diffs.size else 0.0,
                "spike_time_err_ms_mean": float(diffs.mean()) if diffs.size else 0.0,
                "spikes_unmatched_plain": un_a, "spikes_unmatched_surrogate": un_b,
                "checked": checked, "flagged": flagged, "guarded": guarded,
                "plain_cell_macro_steps": plain_cells}

    surr = run()
    hold = run(mode="plain_hold")
    nofb = run(sample_every=0, v_max=1e30, z_max=0.0, ca_max=1e30)
    log("surrogate leg: surrogate and ablations done")
    return {
        "dt_steps": SURR_DT, "macro_steps": SURR_DT // 4,
        "plain_ms": t_plain, "surrogate_ms": surr["ms"],
        "speedup": t_plain / surr["ms"],
        "rmse_mv": surr["rmse_mv"],
        "spike_time_err_ms": surr["spike_time_err_ms_max"],
        "spikes_plain": int(ca.sum()), "spikes_surrogate": surr["spikes"],
        "surrogate": surr,
        "ablation_held_gap_no_mlp": {"speedup": t_plain / hold["ms"], **hold},
        "ablation_mlp_no_fallback": {"speedup": t_plain / nofb["ms"], **nofb},
        "mlp_gain_over_held_gap": hold["ms"] / surr["ms"],
        "training": {**rep, "wall_s": train_wall},
    }


def spiking_accuracy_leg(params, norm, infoli, log, steps=2000):
    """The surrogate where cells fire: the 65,536-cell network under the
    paper's validation pulse (Section 3: about 500 steps, here 6 uA/cm^2
    during steps [400, 900)), plain method against the surrogate for `steps`
    time steps; RMSE at every 100 dt and spike times matched per cell."""
    net = I.config4()
    net.pulses = [I.Pulse(400, 900, 6.0)]
    x0 = infoli.initial_state(net)
    sim = infoli.Simulator(net, init_states=[x0], step_mode="graph", graph_chunk=100)
    V = [I.IDX_VD, I.IDX_VS, I.IDX_VA]
    every, ref = 25, []
    for _ in range(steps // 100):
        sim.step(4 * every)
        ref.append(sim.read_state(0)[V])
    ca, ta = sim.read_spikes(0)
    sim.write_state(0, x0, 0)
    sim.clear_spikes()
    sim.surrogate_set(params, norm)
    sq, n, plain_cells, guarded = 0.0, 0, 0, 0
    for k in range(steps // 100):
        r = sim.step_surrogate(every)
        plain_cells += r["plain_cell_macro_steps"]
        guarded += r["guarded"]
        d = (sim.read_state(0)[V] - ref[k]).astype(np.float64)
        sq += float((d * d).sum())
        n += d.size
    cb, tb = sim.read_spikes(0)
    diffs, un_a, un_b = match_spikes(ca, ta, cb, tb, sim.spike_cap)
    sim.close()
    log("spiking accuracy leg done")
    return {"pulse": "6 uA/cm^2, steps [400, 900)", "dt_steps": steps,
            "rmse_mv": float(np.sqrt(sq / n)), "spikes_plain": int(ca.sum()), "spikes_surrogate": int(cb.sum()),
            "cells_spiking_plain": int((ca > 0).sum()),
            "spike_time_err_ms_max": float(diffs.max()) if diffs.size else None,
            "spike_time_err_ms_mean": float(diffs.mean()) if diffs.size else None,
            "spikes_matched": int(diffs.size), "spikes_unmatched_plain": un_a,
            "spikes_unmatched_surrogate": un_b, "plain_cell_macro_steps": plain_cells, "guarded": guarded}


def run_c4(nets, desc, steps, warmup, args, torch, infoli):
    """The 65,536-cell network of mean degree 1,000: the plain step timed
    over exactly `steps` steps, every one a graph replay (graphs captured at
    init); then the surrogate comparison at its full length."""
    net = nets[0]
    log = (lambda m: print(m, file=sys.stderr, flush=True))
    x0 = infoli.initial_state(net)
    chunk = graph_chunk_for(steps)
    stream = torch.cuda.current_stream().cuda_stream
    mode = "launch" if args.mode == "launch" else "graph"
    sim = infoli.Simulator(net, init_states=[x0], stream=stream, step_mode=mode, graph_chunk=chunk,
                           csr_path=args.csr_path)
    info = sim.info()
    paths = [sim.gap_path(0)[0]]
    log(f"c4: context ready ({info['n_tiles']} tiles, graph chunk {chunk})")
    wall, dev_ms = time_plain(sim, steps, warmup, torch)
    launch_s = dev_ms * 1e-3 / steps
    kernel = step_kernel_name(info, nets, paths)
    cells, pairs = net.n, net.pairs_per_step()
    out = {
        "metric": "cell-steps/sec and gap pairs/sec at 1 MI355X; surrogate vs plain speedup at 1 mV RMSE",
        "value": cells * steps / wall,
        "unit": "cell-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c4: {desc}", "cells": cells, "gap_pairs_per_step": pairs,
                   "step_mode": mode, "graph_chunk": chunk, **tuned_config(info, sim, nets)},
        "gap_pairs_per_s": pairs * steps / wall,
        "device_ms_per_step": dev_ms / steps,
        "roofline": roofline(nets, launch_s, kernel, paths),
        "stability": stability(nets),
    }
    out["roofline"]["traffic_key"] = traffic_key("c4", kernel, paths, info)
    out["roofline"]["traffic"] = measured_traffic(out["roofline"]["traffic_key"])
    log(f"c4: plain {dev_ms / steps * 1e3:.2f} us/step")
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg(net, x0, sim, torch, infoli, log, args.load_surrogate,
                                         args.save_surrogate)
        params, norm = sim.surrogate_get()
        out["surrogate"]["spiking_validation_pulse"] = spiking_accuracy_leg(params, norm, infoli, log)
    sim.close()
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
    if args.rt_case:
        unknown = sorted(set(args.rt_case) - set(cases))
        if unknown:
            raise SystemExit(f"--rt-case: unknown {unknown}; one of {cases}")
        cases = [c for c in cases if c in args.rt_case]
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


# Table 4's scenario (Section 3.2): per network size a batch of five
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
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="auto", choices=["graph", "launch", "auto", "persistent"])
    ap.add_argument("--graph-chunk", type=int, default=100)
    ap.add_argument("--csr-path", type=int, default=0,
                    help="force a CSR gap path (the library's csr_path option; 0: tuned)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="c4: the plain step only")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--rt-sweep", action="store_true",
                    help="only run the real-time size sweep (largest network per use case within the budget)")
    ap.add_argument("--rt-budget-us", type=float, default=50.0)
    ap.add_argument("--rt-case", action="append", default=[],
                    help="with --rt-sweep: only this use case (repeatable), e.g. 'RGJ 100%%'")
    ap.add_argument("--paper-batches", action="store_true",
                    help="only run Table 4's experiment batches (per size, five densities)")
    ap.add_argument("--copy-probe-mb", type=float, default=0.0,
                    help="only run a device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--save-surrogate", default=None, metavar="NPZ",
                    help="c4: write the trained surrogate's weights and normalisation here")
    ap.add_argument("--load-surrogate", default=None, metavar="NPZ",
                    help="c4: use these weights and normalisation instead of training")
    ap.add_argument("--ingest-traffic", default=None, metavar="DIR",
                    help="only read the rocprofv3 FETCH_SIZE/WRITE_SIZE runs under DIR into the traffic file")
    args = ap.parse_args()
    if args.ingest_traffic:
        ingest_traffic(args.ingest_traffic)
        return
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
    if args.workload == "c4":
        run_c4(nets, desc, steps, warmup, args, torch, infoli)
        return
    if args.workload == "valid120k":
        run_validation(nets, desc, steps, warmup, args, torch, infoli)
        return
    x0s = [infoli.initial_state(n) for n in nets]
    stream = torch.cuda.current_stream().cuda_stream
    mode = args.mode
    chunk = args.graph_chunk
    if mode == "auto" and not (len(nets) == 1 and nets[0].n <= 1024):
        # every timed step a graph replay: chunks that divide the step count,
        # captured at init (a lone network of <= 1,024 cells stays in the
        # library's automatic choice, which times the persistent kernel)
        mode, chunk = "graph", graph_chunk_for(steps, args.graph_chunk)
    sim = infoli.Simulator(nets, init_states=x0s, stream=stream, step_mode=mode, graph_chunk=chunk,
                           csr_path=args.csr_path)
    info = sim.info()
    paths = [sim.gap_path(k)[0] for k in range(len(nets))]
    wall, dev_ms = time_plain(sim, steps, warmup, torch)
    tuned = tuned_config(info, sim, nets)
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
                   "gap_pairs_per_step": pairs, "step_mode": mode, "graph_chunk": chunk, **tuned},
        "gap_pairs_per_s": pairs * steps / wall,
        "device_ms_per_step": dev_ms / steps,
        "roofline": roofline(nets, launch_s, step_kernel_name(info, nets, paths), paths),
        "stability": stability(nets),
    }
    out["roofline"]["traffic_key"] = traffic_key(args.workload, step_kernel_name(info, nets, paths), paths, info)
    out["roofline"]["traffic"] = measured_traffic(out["roofline"]["traffic_key"])
    if args.workload in NO_CPU_BASELINE:
        out["cpu_baseline"] = None
        out["cpu_baseline_note"] = NO_CPU_BASELINE[args.workload]
    elif not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nets, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
