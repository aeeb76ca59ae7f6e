"""Python access to the plain CPU oracle (oracle/infoli_oracle.c) and the
numpy MLP oracle (oracle/mlp.py).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use it; the GPU library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

CONN = {"none": 0, "uniform": 1, "dense": 2, "csr": 3}
N_STATE = 14
N_PARAMS = 20


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no fast-math, no FP contraction)."""
    src = [os.path.join(HERE, "infoli_oracle.c"), os.path.join(HERE, "oracle_body.inc")]
    if force or not os.path.exists(LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(LIB_PATH) for s in src):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-fPIC", "-shared", "-o", tmp, src[0], "-lm"]
        subprocess.check_call(cmd, cwd=HERE)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _make_net_struct(real):
    P = ctypes.POINTER
    return type("OrcNet_" + real.__name__, (ctypes.Structure,), {"_fields_": [
        ("n", ctypes.c_int32), ("conn", ctypes.c_int32), ("g", real), ("dt", real),
        ("w_dense", P(real)), ("row_ptr", P(ctypes.c_int64)), ("col", P(ctypes.c_int32)),
        ("w_csr", P(real)), ("params", P(real)), ("bias", P(real)),
        ("n_pulses", ctypes.c_int32), ("pulse_n0", P(ctypes.c_int64)),
        ("pulse_n1", P(ctypes.c_int64)), ("pulse_c0", P(ctypes.c_int32)),
        ("pulse_c1", P(ctypes.c_int32)), ("pulse_amp", P(real)),
        ("i_stream", P(real)), ("i_stream_steps", ctypes.c_int64),
        ("reverse_j", ctypes.c_int32), ("sgj", ctypes.c_int32), ("cell_params", P(real))]})


_NET64 = _make_net_struct(ctypes.c_double)
_NET32 = _make_net_struct(ctypes.c_float)
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Oracle:
    """The plain method in one precision ('f64' or 'f32')."""

    def __init__(self, precision: str = "f64"):
        assert precision in ("f64", "f32")
        self.precision = precision
        self.np_real = np.float64 if precision == "f64" else np.float32
        self.c_real = ctypes.c_double if precision == "f64" else ctypes.c_float
        self.Net = _NET64 if precision == "f64" else _NET32
        L = lib()
        self._rest = getattr(L, "orc_rest_" + precision)
        self._gap = getattr(L, "orc_gap_" + precision)
        self._iapp = getattr(L, "orc_iapp_" + precision)
        self._rhs = getattr(L, "orc_rhs_" + precision)
        self._run = getattr(L, "orc_run_" + precision)
        self._rest.argtypes = [ctypes.POINTER(self.c_real), self.c_real,
                               ctypes.POINTER(self.c_real)]
        self._rhs.argtypes = [ctypes.POINTER(self.c_real)] * 2 + [self.c_real] * 2 + [
            ctypes.POINTER(self.c_real)]
        self._rhs.restype = None
        self._run.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                              ctypes.POINTER(self.c_real), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(self.c_real), ctypes.c_int32,
                              ctypes.POINTER(self.c_real), ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_int32]

    # ------------------------------------------------------------ helpers
    def _arr(self, a):
        return None if a is None else np.ascontiguousarray(a, dtype=self.np_real)

    def _struct(self, net, reverse_j=False, i_stream=None):
        keep = {}
        R = self.np_real
        keep["params"] = np.ascontiguousarray(net.params, dtype=R)
        keep["w_dense"] = self._arr(net.w_dense)
        keep["row_ptr"] = None if net.row_ptr is None else np.ascontiguousarray(net.row_ptr, np.int64)
        keep["col"] = None if net.col is None else np.ascontiguousarray(net.col, np.int32)
        keep["w_csr"] = self._arr(net.w_csr)
        keep["bias"] = self._arr(net.bias)
        np_ = len(net.pulses)
        keep["p_n0"] = np.array([p.step_begin for p in net.pulses] or [0], np.int64)
        keep["p_n1"] = np.array([p.step_end for p in net.pulses] or [0], np.int64)
        keep["p_c0"] = np.array([p.cell_begin for p in net.pulses] or [0], np.int32)
        keep["p_c1"] = np.array([(net.n if p.cell_end < 0 else p.cell_end)
                                 for p in net.pulses] or [0], np.int32)
        keep["p_a"] = np.array([p.amplitude for p in net.pulses] or [0], R)
        keep["i_stream"] = self._arr(i_stream)
        cp = getattr(net, "cell_params", None)
        keep["cell_params"] = None if cp is None else np.ascontiguousarray(cp, dtype=R).reshape(net.n, 20)
        cr = self.c_real
        s = self.Net(n=net.n, conn=CONN[net.conn], g=net.g, dt=net.dt,
                     w_dense=_ptr(keep["w_dense"], cr), row_ptr=_ptr(keep["row_ptr"], ctypes.c_int64),
                     col=_ptr(keep["col"], ctypes.c_int32), w_csr=_ptr(keep["w_csr"], cr),
                     params=_ptr(keep["params"], cr), bias=_ptr(keep["bias"], cr),
                     n_pulses=np_, pulse_n0=_ptr(keep["p_n0"], ctypes.c_int64),
                     pulse_n1=_ptr(keep["p_n1"], ctypes.c_int64),
                     pulse_c0=_ptr(keep["p_c0"], ctypes.c_int32),
                     pulse_c1=_ptr(keep["p_c1"], ctypes.c_int32),
                     pulse_amp=_ptr(keep["p_a"], cr),
                     i_stream=_ptr(keep["i_stream"], cr),
                     i_stream_steps=0 if i_stream is None else int(i_stream.shape[0]),
                     reverse_j=1 if reverse_j else 0,
                     sgj=1 if getattr(net, "gap", "rgj") == "sgj" else 0,
                     cell_params=_ptr(keep["cell_params"], cr))
        return s, keep

    # ------------------------------------------------------------ API
    def rest(self, params=None, v0: float = -60.0) -> np.ndarray:
        from paper_1612_01501_amd.inputs import DEFAULT_PARAMS
        p = np.ascontiguousarray(DEFAULT_PARAMS if params is None else params, self.np_real)
        x = np.zeros(N_STATE, self.np_real)
        self._rest(_ptr(p, self.c_real), self.c_real(v0), _ptr(x, self.c_real))
        return x

    def initial_state(self, net, v0: float = -60.0) -> np.ndarray:
        """Rest state for every cell (each cell's own, when the network has
        per-cell parameters) plus the network's voltage jitter, [S][n]."""
        cp = getattr(net, "cell_params", None)
        if cp is None:
            r = self.rest(net.params, v0).astype(np.float64)
            x = np.repeat(r[:, None], net.n, axis=1)
        else:
            x = np.stack([self.rest(cp[i], v0).astype(np.float64) for i in range(net.n)], axis=1)
        if net.jitter is not None:
            for row, v in enumerate((0, 5, 11)):
                x[v] += net.jitter[row]
        return x.astype(self.np_real)

    def rhs(self, x14, igap=0.0, iapp=0.0, params=None) -> np.ndarray:
        from paper_1612_01501_amd.inputs import DEFAULT_PARAMS
        p = np.ascontiguousarray(DEFAULT_PARAMS if params is None else params, self.np_real)
        x = np.ascontiguousarray(x14, self.np_real)
        dx = np.zeros(N_STATE, self.np_real)
        self._rhs(_ptr(p, self.c_real), _ptr(x, self.c_real), self.c_real(igap),
                  self.c_real(iapp), _ptr(dx, self.c_real))
        return dx

    def gap(self, net, vd, reverse_j=False) -> np.ndarray:
        s, keep = self._struct(net, reverse_j)
        v = np.ascontiguousarray(vd, self.np_real)
        out = np.zeros(net.n, self.np_real)
        rc = self._gap(ctypes.byref(s), _ptr(v, self.c_real), _ptr(out, self.c_real))
        assert rc == 0
        return out

    def iapp(self, net, step: int, i_stream=None) -> np.ndarray:
        s, keep = self._struct(net, i_stream=i_stream)
        out = np.zeros(net.n, self.np_real)
        self._iapp.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(self.c_real)]
        self._iapp(ctypes.byref(s), step, _ptr(out, self.c_real))
        return out

    def run(self, net, steps: int, x0: Optional[np.ndarray] = None, step0: int = 0,
            trace_every: int = 0, trace_cells: int = 0, spike_cap: int = 64,
            threads: int = 0, reverse_j: bool = False, i_stream=None):
        """Run `steps` steps from x0 (default: initial_state(net)).

        Returns dict(x=[S][n] final state, counts=[n] int32, times=[n][cap] ms,
        trace=[m][S][trace_cells] or None).
        """
        x = self.initial_state(net) if x0 is None else np.array(x0, dtype=self.np_real, copy=True)
        x = np.ascontiguousarray(x)
        assert x.shape == (N_STATE, net.n)
        s, keep = self._struct(net, reverse_j, i_stream)
        counts = np.zeros(net.n, np.int32)
        times = np.full((net.n, max(spike_cap, 1)), np.nan, self.np_real)
        trace = None
        if trace_every > 0:
            m = steps // trace_every
            trace = np.zeros((m, N_STATE, trace_cells), self.np_real)
        rc = self._run(ctypes.byref(s), step0, steps, _ptr(x, self.c_real),
                       _ptr(counts, ctypes.c_int32), _ptr(times, self.c_real), spike_cap,
                       _ptr(trace, self.c_real) if trace is not None else None,
                       trace_every, trace_cells, threads)
        assert rc == 0, rc
        return {"x": x, "counts": counts, "times": times, "trace": trace}


def max_threads() -> int:
    return int(lib().orc_max_threads())
