"""Host-side checks of the C ABI: the library loads, exports every entry point
the header declares, and its host-only functions and spec validation behave
(no device work is started here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1612_01501_amd import infoli, inputs as I

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "infoli.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(infoli_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = infoli.lib()
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
    assert set(infoli.EXPORTS) == set(names)


def test_gap_path_names_follow_header_enum():
    """The binding's gap-path names are indexed by the header's
    infoli_gap_path codes."""
    text = open(HEADER).read()
    body = re.search(r"typedef enum infoli_gap_path \{(.*?)\} infoli_gap_path;", text, flags=re.S).group(1)
    codes = {name.lower(): int(v) for name, v in re.findall(r"INFOLI_PATH_([A-Z_0-9]+)\s*=\s*(\d+)", body)}
    assert sorted(codes.values()) == list(range(len(infoli.GAP_PATH)))
    for name, v in codes.items():
        assert infoli.GAP_PATH[v] == name, (name, v)


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors have the C compiler's sizes and field offsets."""
    src = tmp_path / "sz.c"
    exe = tmp_path / "sz"
    checks = {"infoli_pulse": infoli.Pulse, "infoli_network_spec": infoli.NetworkSpec,
              "infoli_options": infoli.Options, "infoli_info": infoli.Info,
              "infoli_train_cfg": infoli.TrainCfg, "infoli_train_report": infoli.TrainReport,
              "infoli_drift_cfg": infoli.DriftCfg, "infoli_drift_report": infoli.DriftReport}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in checks.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    import subprocess
    subprocess.check_call(["gcc", "-std=c99", "-o", str(exe), str(src)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    k = 0
    for cname, py in checks.items():
        assert vals[k] == ctypes.sizeof(py), cname
        k += 1
        for f, _ in py._fields_:
            assert vals[k] == getattr(py, f).offset, (cname, f)
            k += 1


def test_default_params_match_input_table():
    np.testing.assert_array_equal(infoli.default_params(), I.DEFAULT_PARAMS.astype(np.float32))


def test_rest_state_matches_oracle(o64, o32):
    lib_rest = infoli.rest_state().astype(np.float64)
    np.testing.assert_allclose(lib_rest, o64.rest(), rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(lib_rest, o32.rest().astype(np.float64), rtol=2e-6, atol=1e-9)
    for v0 in (-70.0, -8.5, -25.0):
        np.testing.assert_allclose(infoli.rest_state(v0=v0).astype(np.float64), o64.rest(v0=v0),
                                   rtol=5e-6, atol=1e-9)


def test_state_names_and_errors():
    L = infoli.lib()
    names = [L.infoli_state_var_name(v).decode() for v in range(14)]
    assert names == list(I.STATE_NAMES)
    assert L.infoli_state_var_name(14) is None
    assert L.infoli_state_var_name(-1) is None
    assert L.infoli_default_params(None) == 1
    assert b"NULL" in L.infoli_last_error(None)
    p = ctypes.c_int32(-1)
    assert L.infoli_get_gap_path(None, 0, ctypes.byref(p), None) == 1
    assert p.value == -1


def _init_status(net, **kw):
    """Run infoli_init on a spec that must fail validation (before any device
    call) and return the status and message."""
    h = infoli._SpecHolder(net, init_state=np.zeros((14, net.n), np.float32) - 60.0)
    for k, v in kw.items():
        setattr(h.spec, k, v)
    ctx = ctypes.c_void_p(1234)
    st = infoli.lib().infoli_init(ctypes.byref(h.spec), None, ctypes.byref(ctx))
    assert ctx.value is None          # *out is NULL on failure
    return st, infoli.lib().infoli_last_error(None).decode()


def _csr_net(n=5):
    rp, col = I.erdos_renyi_csr(n, 0.6, 3)
    return I.Network(n=n, conn="csr", g=0.04, row_ptr=rp, col=col)


def test_validation_rejects_bad_specs():
    base = I.Network(n=4, conn="uniform", g=0.04)
    assert _init_status(base, n_cells=0)[0] == 1
    assert _init_status(base, dt_ms=0.0)[0] == 1
    assert _init_status(base, dt_ms=float("nan"))[0] == 1
    assert _init_status(base, conn=9)[0] == 1
    assert _init_status(base, g_uniform=float("inf"))[0] == 2
    assert _init_status(base, step0=-1)[0] == 1
    assert _init_status(base, n_pulses=65)[0] == 1


def test_validation_rejects_bad_csr():
    net = _csr_net()
    rp = np.array(net.row_ptr)
    rp_bad = rp.copy()
    rp_bad[2] = rp_bad[3] + 1
    keep = np.ascontiguousarray(rp_bad)
    st, msg = _init_status(net, row_ptr=keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    assert st == 2 and "decreases" in msg
    col = np.array(net.col).copy()
    col[0] = 5
    st, msg = _init_status(net, col=col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert st == 2 and "out of range" in msg
    st, msg = _init_status(net, nnz=int(rp[-1]) + 1)
    assert st == 2
    w = np.full(int(rp[-1]), 0.04, np.float32)
    w[1] = np.nan
    st, msg = _init_status(net, w_csr=w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    assert st == 2 and "non-finite" in msg


def test_validation_rejects_unsorted_or_repeated_columns():
    # the column-block and chunk layouts assume every row strictly ascending
    net = _csr_net(8)
    rp, col = np.array(net.row_ptr), np.array(net.col)
    row = int(np.argmax(np.diff(rp)))                 # a row with >= 2 edges
    b, e = int(rp[row]), int(rp[row + 1])
    assert e - b >= 2
    shuffled = col.copy()
    shuffled[b:e] = shuffled[b:e][::-1]
    st, msg = _init_status(net, col=shuffled.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert st == 2 and "ascending" in msg
    repeated = col.copy()
    repeated[b + 1] = repeated[b]
    st, msg = _init_status(net, col=repeated.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert st == 2 and "ascending" in msg


def test_validation_rejects_bad_dense_and_inputs():
    n = 3
    w = np.ones((n, n), np.float32)
    w[1, 2] = np.inf
    net = I.Network(n=n, conn="dense", w_dense=w)
    assert _init_status(net)[0] == 2
    net = I.Network(n=n, conn="none", bias=np.array([0, np.nan, 0], np.float32))
    assert _init_status(net)[0] == 1
    net = I.Network(n=n, conn="none", pulses=[I.Pulse(10, 5, 1.0)])
    assert _init_status(net)[0] == 1
    net = I.Network(n=n, conn="none", pulses=[I.Pulse(0, 5, 1.0, 0, 4)])
    assert _init_status(net)[0] == 1
    p = I.DEFAULT_PARAMS.copy()
    p[13] = 1.5
    assert _init_status(I.Network(n=n, conn="none", params=p))[0] == 1


def test_validation_rejects_bad_gap_kind():
    net = I.Network(n=3, conn="uniform", g=0.04, gap="sgj")
    st, msg = _init_status(net, gap_kind=2)
    assert st == 1 and "gap_kind" in msg
    st, msg = _init_status(net, reserved0=1)
    assert st == 1 and "reserved0" in msg
    h = infoli._SpecHolder(net, init_state=np.zeros((14, 3), np.float32) - 60.0)
    assert h.spec.gap_kind == 1
    assert infoli._SpecHolder(I.Network(n=3, conn="none"), init_state=np.zeros((14, 3), np.float32)).spec.gap_kind == 0


def test_bad_options_rejected():
    net = I.Network(n=4, conn="none")
    h = infoli._SpecHolder(net, init_state=np.zeros((14, 4), np.float32) - 60.0)
    for kw in ({"graph_chunk": 3}, {"lanes_per_row": 3}, {"tile_rows": 1000},
               {"step_mode": 7}, {"max_spikes_per_cell": -1}, {"wide_threads": 300},
               {"output_ring_steps": -1}):
        opt = infoli.default_options(**kw)
        ctx = ctypes.c_void_p()
        st = infoli.lib().infoli_init(ctypes.byref(h.spec), ctypes.byref(opt), ctypes.byref(ctx))
        assert st in (1, 7), kw
        assert ctx.value is None


def test_mlp_entry_points_validate_arguments():
    L = infoli.lib()
    p = np.zeros(infoli.MLP_PARAMS, np.float32)
    x = np.zeros((10, 16), np.float32)
    y = np.zeros((10, 16), np.float32)
    PF = ctypes.POINTER(ctypes.c_float)
    assert L.infoli_mlp_forward(p.ctypes.data_as(PF), x.ctypes.data_as(PF), 10, y.ctypes.data_as(PF)) == 1
    p[3] = np.nan
    assert L.infoli_mlp_forward(p.ctypes.data_as(PF), x.ctypes.data_as(PF), 16, y.ctypes.data_as(PF)) == 1
    assert L.infoli_mlp_adam_step(None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8) == 1


def test_default_train_and_drift_cfg():
    c = infoli.default_train_cfg()
    assert c.batch % 64 == 0 and c.n_transitions >= 1_000_000 and c.lr > 0
    d = infoli.default_drift_cfg()
    assert d.theta_mv == 0.5 and d.sample_every == 64 and d.hold_steps == 50 and d.v_max == -40.0
    assert d.z_max == 8.0 and c.v_max == d.v_max and c.ca_max == d.ca_max
