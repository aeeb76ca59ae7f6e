"""Host-side checks of bench.py's accounting (no GPU): algorithmic bytes of
small networks by hand, the roofline's bound and units per workload kind,
the step-kernel variant names, and the one-GPU refusal."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1612_01501_amd import inputs as I  # noqa: E402


def _csr(n, edges):
    rows = np.zeros(n + 1, np.int64)
    for i, _ in edges:
        rows[i + 1] += 1
    return np.cumsum(rows), np.array([j for _, j in sorted(edges)], np.int32)


def test_algorithmic_bytes_by_hand():
    rp, col = _csr(3, [(0, 1), (1, 0), (1, 2), (2, 1)])
    csr = I.Network(n=3, conn="csr", g=0.04, row_ptr=rp, col=col)
    # 116 B per cell (14 state floats in and out, bias), 2 B per uint16
    # column, 8 B per row pointer
    assert bench.algorithmic_bytes([csr]) == 116 * 3 + 2 * 4 + 8 * 3
    csr_w = I.Network(n=3, conn="csr", row_ptr=rp, col=col, w_csr=np.full(4, 0.04, np.float32))
    assert bench.algorithmic_bytes([csr_w]) == 116 * 3 + (2 + 4) * 4 + 8 * 3
    dense = I.Network(n=2, conn="dense", w_dense=np.ones((2, 2), np.float32))
    assert bench.algorithmic_bytes([dense]) == 116 * 2 + 4 * 4
    assert bench.algorithmic_bytes([I.Network(n=5, conn="uniform", g=0.1)]) == 116 * 5
    assert bench.algorithmic_bytes([I.Network(n=7, conn="none")]) == 116 * 7
    # a network on the coupling bitmap streams one bit per (row, column)
    # pair, rows of whole 32-bit words, instead of columns and row pointers
    assert bench.algorithmic_bytes([csr], ["csr_bitmap"]) == 116 * 3 + 4 * 3 * 1
    big = I.Network(n=40, conn="csr", g=0.04, row_ptr=np.zeros(41, np.int64), col=np.zeros(0, np.int32))
    assert bench.algorithmic_bytes([big], ["csr_bitmap"]) == 116 * 40 + 4 * 40 * 2
    assert bench.algorithmic_bytes([csr], ["csr_chunked"]) == bench.algorithmic_bytes([csr])


def test_roofline_bound_per_workload_kind():
    uni = bench.roofline([I.Network(n=100, conn="uniform", g=0.1)], 1e-6)
    assert uni["bound"] == "alu" and uni["unit"] == "Gpair/s"
    assert uni["achieved"] == pytest.approx(100 * 100 / 1e-6 / 1e9)
    assert uni["frac"] == pytest.approx(uni["achieved"] / uni["peak"])
    assert uni["frac_vs_exp_shared_minimum"] < uni["frac"]
    rp, col = _csr(3, [(0, 1), (1, 0)])
    csr = bench.roofline([I.Network(n=3, conn="csr", g=0.04, row_ptr=rp, col=col)], 1e-6)
    assert csr["bound"] == "hbm" and csr["unit"] == "GB/s" and csr["peak"] == 8000.0
    assert csr["achieved"] == pytest.approx(bench.algorithmic_bytes(
        [I.Network(n=3, conn="csr", g=0.04, row_ptr=rp, col=col)]) / 1e-6 / 1e9)
    sgj = bench.roofline([I.Network(n=100, conn="uniform", g=0.1, gap="sgj")], 1e-6)
    assert sgj["bound"] == "hbm" and "alu_frac" in sgj
    ngj = bench.roofline([I.Network(n=64, conn="none")], 1e-6)
    assert ngj["alu_slots_per_cell_step"] == bench.CELL_SLOTS
    mixed = bench.roofline([I.Network(n=10, conn="uniform", g=0.1),
                            I.Network(n=3, conn="csr", g=0.04, row_ptr=rp, col=col)], 1e-6)
    assert mixed["bound"] == "alu" and mixed["unit"] == "T lane-slots/s"
    # composite: per network the larger of bytes at the HBM peak and slots
    # (compartment updates and pair work) at the lane-slot peak, summed
    u = (bench.UNIFORM_SLOTS_PER_PAIR * 10 * 10 + bench.CELL_SLOTS * 10) / bench.LANE_SLOTS_PER_S
    c_bytes = (116 * 3 + 2 * 2 + 8 * 3) / 8e12
    c_slots = (bench.CSR_SLOTS_PER_EDGE * 2 + bench.CELL_SLOTS * 3) / bench.LANE_SLOTS_PER_S
    assert mixed["slots_per_launch"] == pytest.approx(
        bench.UNIFORM_SLOTS_PER_PAIR * 100 + bench.CELL_SLOTS * 13 + bench.CSR_SLOTS_PER_EDGE * 2)
    assert mixed["composite_roofline_us"] == pytest.approx((max(116 * 10 / 8e12, u) + max(c_bytes, c_slots)) * 1e6)
    assert mixed["composite_frac"] == pytest.approx(mixed["composite_roofline_us"] * 1e-6 / 1e-6)


def test_csr_roofline_takes_the_larger_bound():
    """All-CSR launches: bound = the larger of bytes at the HBM peak and issue
    slots at the lane-slot peak, each network counted in its path's form."""
    n = 128
    edges = [(i, j) for i in range(n) for j in range(n) if i != j and (i + j) % 2 == 1]
    rp, col = _csr(n, edges)
    net = I.Network(n=n, conn="csr", g=0.04, row_ptr=rp, col=col)
    launch = 1e-6
    gath = bench.roofline([net], launch, paths=["csr_gather"])
    b_g = 116 * n + 2 * len(edges) + 8 * n
    s_g = bench.CELL_SLOTS * n + bench.CSR_SLOTS_PER_EDGE * len(edges)
    assert gath["algorithmic_bytes_per_launch"] == b_g and gath["slots_per_launch"] == pytest.approx(s_g)
    bit = bench.roofline([net], launch, paths=["csr_bitmap"])
    b_b = 116 * n + 4 * n * ((n + 31) // 32)
    s_b = bench.CELL_SLOTS * n + bench.BITMAP_SLOTS_PER_PAIR * n * n
    assert bit["algorithmic_bytes_per_launch"] == b_b and bit["slots_per_launch"] == pytest.approx(s_b)
    for r, b, sl in ((gath, b_g, s_g), (bit, b_b, s_b)):
        t_hbm, t_alu = b / 8e12, sl / bench.LANE_SLOTS_PER_S
        assert r["hbm_frac"] == pytest.approx(t_hbm / launch) and r["alu_frac"] == pytest.approx(t_alu / launch)
        assert r["bound"] == ("alu" if t_alu > t_hbm else "hbm")
        assert r["frac"] == pytest.approx(max(t_hbm, t_alu) / launch)
    assert bit["bound"] == "alu" and bit["unit"] == "T lane-slots/s" and bit["gap_paths"] == ["csr_bitmap"]
    # simplified gap junctions cost fewer slots per edge
    sgj = I.Network(n=n, conn="csr", g=0.04, row_ptr=rp, col=col, gap="sgj")
    assert bench.slots_of(sgj) == pytest.approx(bench.CELL_SLOTS * n + bench.SGJ_SLOTS_PER_EDGE * len(edges))


def test_issue_slot_peak_is_the_published_fp32_peak():
    """One lane-slot per FMA lane: the lane-slot peak is MI355X's FP32 vector
    peak (157.3 TFLOP/s, two flops per FMA); a transcendental costs the
    measured 3.3 slots, in every slot count that has one."""
    assert bench.LANE_SLOTS_PER_S == pytest.approx(157.3e12 / 2, rel=1e-3)
    e = bench.EXP_SLOTS
    assert e == pytest.approx(3.3)
    assert bench.UNIFORM_SLOTS_PER_PAIR == pytest.approx(3 + e)
    assert bench.CSR_SLOTS_PER_EDGE == pytest.approx(7 + e)
    assert bench.BITMAP_SLOTS_PER_PAIR == pytest.approx(5 + e)
    assert bench.CELL_SLOTS == pytest.approx(239 + 39 * e)


def test_step_kernel_variant_names():
    info = {"step_mode": 0, "n_tiles_wide": 0, "n_tiles": 4}
    rp, col = _csr(3, [(0, 1), (1, 0)])
    plain = I.Network(n=3, conn="csr", g=0.04, row_ptr=rp, col=col)
    weighted = I.Network(n=3, conn="csr", row_ptr=rp, col=col, w_csr=np.ones(2, np.float32))
    assert bench.step_kernel_name(info, [I.Network(n=8, conn="none")]) == "infoli::k_step<256, 1>"
    assert bench.step_kernel_name(info, [plain]) == "infoli::k_step<256, 2>"
    assert bench.step_kernel_name(info, [weighted]) == "infoli::k_step<256, 0>"
    assert bench.step_kernel_name({**info, "n_tiles_wide": 4}, [plain]) == "infoli::k_step<1024, 2>"
    assert bench.step_kernel_name({**info, "n_tiles_wide": 4, "wide_threads": 512}, [plain]) == "infoli::k_step<512, 2>"
    assert bench.step_kernel_name({**info, "step_mode": 3}, [plain]) == "infoli::k_persist"


def test_measured_traffic_needs_matching_sources():
    assert bench.measured_traffic("no-such-workload") is None
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if os.path.exists(path):
        d = json.load(open(path))
        for w, v in d.items():
            if w == "calibration":
                continue
            got = bench.measured_traffic(w)
            if v.get("kernel_sources_sha256") == bench.kernel_source_hash():
                assert got == v["bytes_per_launch"]
            else:
                assert got is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_graph_chunk_divides_the_timed_steps():
    assert bench.graph_chunk_for(20) == 20
    assert bench.graph_chunk_for(2000) == 100
    assert bench.graph_chunk_for(1000) == 100
    assert bench.graph_chunk_for(30) == 30
    assert bench.graph_chunk_for(35) == 2           # no even divisor: pairs of steps
    for k in (20, 2000, 4000, 10000, 120000, 42):
        c = bench.graph_chunk_for(k)
        assert c % 2 == 0 and c >= 2 and (k % c == 0 or c == 2)


def test_spike_matching_by_nearest_time():
    cap = 4
    ca = np.array([2, 0, 1], np.int32)
    ta = np.array([[10.0, 20.0, 0, 0], [0, 0, 0, 0], [5.0, 0, 0, 0]], np.float32)
    cb = np.array([2, 1, 0], np.int32)
    tb = np.array([[20.05, 9.9, 0, 0], [7.0, 0, 0, 0], [0, 0, 0, 0]], np.float32)
    d, un_a, un_b = bench.match_spikes(ca, ta, cb, tb, cap)
    assert sorted(np.round(d, 4)) == [0.05, 0.1]
    assert un_a == 1 and un_b == 1


def test_stability_is_gershgorin_of_the_laplacian():
    rp, col = _csr(3, [(0, 1), (0, 2), (1, 0), (2, 0)])
    net = I.Network(n=3, conn="csr", g=0.5, row_ptr=rp, col=col)
    s = bench.stability([net])
    assert s["dt_lambda_max_gershgorin"] == pytest.approx(0.05 * 2 * 2 * 0.5)
    uni = I.Network(n=96, conn="uniform", g=0.04)
    s = bench.stability([uni, net])
    assert s["dt_lambda_max_gershgorin"] == pytest.approx(0.05 * 2 * 95 * 0.04)
    assert s["euler_stable"] and s["networks_above_2"] == 0
    # the 50 % network of 4,096 cells at g = 0.04 is far above the limit
    big = I.Network(n=4, conn="uniform", g=0.04 * 2048 / 3)
    assert not bench.stability([big])["euler_stable"]


def test_traffic_key_names_the_configuration():
    k = bench.traffic_key("c4", "infoli::k_step<1024, 2>", ["csr_chunked"], {"wide_threads": 512})
    assert k == "c4|infoli::k_step<1024, 2>|csr_chunked|wide512"
    assert bench.measured_traffic(k + "x") is None


def test_stream_path_bytes_add_the_row_tags():
    rp, col = _csr(4, [(i, j) for i in range(4) for j in range(4) if i != j])
    net = I.Network(n=4, conn="csr", g=0.04, row_ptr=rp, col=col)
    assert bench.algorithmic_bytes([net], ["csr_stream"]) == bench.algorithmic_bytes([net]) + 12 // 8


def test_stream_kernel_variant_name():
    info = {"step_mode": 0, "n_tiles_wide": 256, "n_tiles": 256, "wide_threads": 1024}
    rp, col = _csr(3, [(0, 1), (1, 0)])
    plain = I.Network(n=3, conn="csr", g=0.04, row_ptr=rp, col=col)
    assert bench.step_kernel_name(info, [plain], ["csr_stream"]) == "infoli::k_step<1024, 3>"
    assert bench.step_kernel_name(info, [plain], ["csr_chunked"]) == "infoli::k_step<1024, 2>"


def _pmc_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    cols = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
            "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
            "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(os.path.join(path, "run_counter_collection.csv"), "w") as fh:
        fh.write(",".join(f'"{c}"' for c in cols) + "\n")
        for d, k, c, v in rows:
            fh.write(f'{d},{d},"Agent 1",1,1,1,64,1,"{k}",64,0,0,8,0,32,"{c}",{v},0,1\n')


def test_traffic_ingest_takes_the_timed_dispatches(tmp_path, monkeypatch):
    """Counter runs -> bytes per launch: the copy calibrates each counter, the
    tuner's earlier dispatches of the same kernel are dropped, and the entry
    lands under the benchmark's traffic key with the source hash."""
    root = str(tmp_path)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", os.path.join(root, "traffic.json"))
    mib = 4
    with open(os.path.join(root, "copy.json"), "w") as fh:
        fh.write(json.dumps({"copy_probe_bytes_read": mib << 20, "copy_probe_bytes_written": mib << 20}) + "\n")
    _pmc_csv(os.path.join(root, "copy_fetch"), [(1, "fill", "FETCH_SIZE", 1.0), (2, "copy", "FETCH_SIZE", 2048.0)])
    _pmc_csv(os.path.join(root, "copy_write"), [(1, "fill", "WRITE_SIZE", 4096.0), (2, "copy", "WRITE_SIZE", 4096.0)])
    kern = "void infoli::k_step<1024, 3>(infoli::StepArgs, float const*, float*, long, int)"
    line = {"steps": 3, "warmup": 1, "roofline": {"kernel": "infoli::k_step<1024, 3>", "traffic_key": "c4|k|p|wide1024",
                                                   "algorithmic_bytes_per_launch": 1000}}
    for k, c, v in (("fetch", "FETCH_SIZE", 10.0), ("write", "WRITE_SIZE", 3.0)):
        with open(os.path.join(root, f"{k}.json"), "w") as fh:
            fh.write("log line\n" + json.dumps(line) + "\n")
        # two tuner dispatches (other sizes), then warmup + timed ones; a second
        # counter of another name is ignored
        rows = [(1, kern, c, 999.0), (2, kern, c, 555.0)] + [(d, kern, c, v) for d in (3, 4, 5, 6)]
        rows += [(7, "other", c, 1e6), (3, kern, "GRBM_COUNT", 7.0)]
        _pmc_csv(os.path.join(root, k), rows)
    bench.ingest_traffic(root)
    table = json.load(open(bench.TRAFFIC_FILE))
    e = table["c4|k|p|wide1024"]
    assert e["dispatches"] == [4, 4]
    assert e["fetch_factor"] == 2.0 and e["write_factor"] == 1.0
    assert e["bytes_per_launch"] == 1024 * (10 * 2 + 3 * 1)
    assert e["kernel_sources_sha256"] == bench.kernel_source_hash()
    assert bench.measured_traffic("c4|k|p|wide1024") == 1024 * 23
    assert bench.measured_traffic("c4|k|p|wide512") is None


def test_unordered_pair_roofline_counts_its_own_work():
    """Each unordered pair once: 7.3 slots per pair of distinct blocks (v_sub,
    v_mul, the exponential, two v_fma), the ordered 6.3 inside each 64-cell
    block, 368 per cell; the two kernels of the step are named."""
    n = 200                                    # 4 blocks: 4 x 64 x 64 own pairs
    net = I.Network(n=n, conn="uniform", g=0.04)
    own = 4 * 64 * 64
    slots = 7.3 * (n * n - own) / 2 + 6.3 * own + bench.CELL_SLOTS * n
    r = bench.roofline([net], 1e-6, "k", ["uniform_sym"])
    assert r["bound"] == "alu" and r["unit"] == "T lane-slots/s"
    assert r["slots_per_launch"] == pytest.approx(slots)
    assert r["frac"] == pytest.approx(slots / 1e-6 / bench.LANE_SLOTS_PER_S)
    assert r["ordered_pair_frac"] == pytest.approx(n * n / 1e-6 / (bench.LANE_SLOTS_PER_S / 6.3))
    assert bench.slots_of(net, "uniform_sym") == pytest.approx(slots)
    info = {"step_mode": 0, "n_tiles_wide": 4, "n_tiles": 4, "wide_threads": 1024}
    assert bench.step_kernel_name(info, [net], ["uniform_sym"]) == \
        "infoli::k_pairs_sym + infoli::k_step<1024, 2>"


def test_voltage_sum_once_keeps_the_byte_roofline():
    """The simplified all-to-all form with the voltage sum taken once per step:
    two kernels named, bound by the bytes of the compartment update (the sum
    adds 8 bytes per 4,096 cells)."""
    net = I.Network(n=40000, conn="uniform", g=0.001, gap="sgj")
    info = {"step_mode": 0, "n_tiles_wide": 0, "n_tiles": 157, "wide_threads": 1024}
    assert bench.step_kernel_name(info, [net], ["uniform_sum"]) == \
        "infoli::k_vsum + infoli::k_step<256, 2>"
    r = bench.roofline([net], 1e-5, "k", ["uniform_sum"])
    assert r["bound"] == "hbm"
    assert r["algorithmic_bytes_per_launch"] == bench.algorithmic_bytes([net], ["uniform"])


def test_source_hash_ignores_comments_only():
    """The traffic records are keyed by the kernel sources' code: comments and
    layout do not count, string literals and code do."""
    a = 'int x = 1; // one\n/* two */ const char* s = "a // b";\n'
    b = 'int  x = 1;\n\n const char* s = "a // b"; // other words\n'
    c = 'int x = 2; const char* s = "a // b";'
    d = 'int x = 1; const char* s = "a /* b";'
    assert bench.code_of(a) == bench.code_of(b)
    assert bench.code_of(a) != bench.code_of(c)
    assert bench.code_of(a) != bench.code_of(d)
    assert "a // b" in bench.code_of(a)
