"""ctypes binding of libinfoli (include/infoli.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; nothing here
computes model quantities. PyTorch, when used, only supplies device memory
and streams (pass ``stream=torch.cuda.current_stream().cuda_stream``).
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Union

import numpy as np

from . import inputs as _inputs

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinfoli.so")

OK = 0
STATUS = {0: "OK", 1: "E_INVALID_ARG", 2: "E_BAD_GRAPH", 3: "E_OUT_OF_MEMORY", 4: "E_DEVICE",
          5: "E_NUMERIC", 6: "E_STATE", 7: "E_UNSUPPORTED"}
CONN = {"none": 0, "uniform": 1, "dense": 2, "csr": 3}
MODE = {"auto": 0, "launch": 1, "graph": 2, "persistent": 3}
NUM_STATE = 14
NUM_PARAMS = 20

# Entry points declared in include/infoli.h (checked by the host tests).
EXPORTS = (
    "infoli_default_options", "infoli_default_params", "infoli_rest_state", "infoli_init",
    "infoli_batch_init", "infoli_step", "infoli_sync", "infoli_read_state",
    "infoli_read_state_device", "infoli_write_state", "infoli_read_gap_current",
    "infoli_read_spikes", "infoli_clear_spikes", "infoli_output_copy_async", "infoli_output_wait",
    "infoli_get_info", "infoli_get_gap_path", "infoli_last_step_ms",
    "infoli_state_var_name", "infoli_last_error", "infoli_destroy",
    "infoli_default_train_cfg", "infoli_default_drift_cfg", "infoli_surrogate_train",
    "infoli_surrogate_get", "infoli_surrogate_set", "infoli_step_surrogate",
    "infoli_mlp_forward", "infoli_mlp_loss_grad", "infoli_mlp_adam_step",
    "infoli_mlp_loss_grad_noalloc",
)
MLP_PARAMS = 20752
SURROGATE_MODE = {"mlp": 0, "plain_hold": 1}


class InfoliError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Pulse(ctypes.Structure):
    _fields_ = [("step_begin", ctypes.c_int64), ("step_end", ctypes.c_int64),
                ("amplitude", ctypes.c_float), ("cell_begin", ctypes.c_int32),
                ("cell_end", ctypes.c_int32)]


_PF = ctypes.POINTER(ctypes.c_float)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PI32 = ctypes.POINTER(ctypes.c_int32)


class NetworkSpec(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32), ("dt_ms", ctypes.c_float), ("conn", ctypes.c_int32),
                ("g_uniform", ctypes.c_float), ("w_dense", _PF), ("row_ptr", _PI64),
                ("col", _PI32), ("w_csr", _PF), ("nnz", ctypes.c_int64), ("params", _PF),
                ("init_state", _PF), ("i_bias", _PF), ("pulses", ctypes.POINTER(Pulse)),
                ("n_pulses", ctypes.c_int32), ("i_stream", _PF),
                ("i_stream_steps", ctypes.c_int64), ("step0", ctypes.c_int64),
                ("gap_kind", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("cell_params", ctypes.POINTER(ctypes.c_float))]


class Options(ctypes.Structure):
    _fields_ = [("hip_stream", ctypes.c_void_p), ("step_mode", ctypes.c_int32),
                ("graph_chunk", ctypes.c_int32), ("max_spikes_per_cell", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("lanes_per_row", ctypes.c_int32),
                ("check_finite", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("csr_path", ctypes.c_int32), ("output_ring_steps", ctypes.c_int32),
                ("wide_threads", ctypes.c_int32), ("pair_path", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int32), ("total_cells", ctypes.c_int64),
                ("pairs_per_step", ctypes.c_int64), ("step", ctypes.c_int64),
                ("step_mode", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("lanes_per_row", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("tuned", ctypes.c_int32),
                ("tune_cached", ctypes.c_int32), ("n_tiles_wide", ctypes.c_int32),
                ("n_bitmap", ctypes.c_int32), ("n_blocked", ctypes.c_int32),
                ("wide_threads", ctypes.c_int32), ("n_stream", ctypes.c_int32),
                ("tune_mode", ctypes.c_int32), ("stream_round", ctypes.c_int32), ("n_sym", ctypes.c_int32)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("n_transitions", ctypes.c_int64), ("n_trajectories", ctypes.c_int32),
                ("burn_in", ctypes.c_int32), ("batch", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("lr_min", ctypes.c_float), ("v_max", ctypes.c_float),
                ("bias_sd", ctypes.c_float), ("gap_sd", ctypes.c_float),
                ("gap_rho", ctypes.c_float), ("pulse_p", ctypes.c_float), ("pulse_lo", ctypes.c_float),
                ("pulse_hi", ctypes.c_float), ("pulse_len", ctypes.c_int32),
                ("ca_max", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("init_params", _PF)]


class TrainReport(ctypes.Structure):
    _fields_ = [("n_transitions", ctypes.c_int64), ("steps", ctypes.c_int32),
                ("loss_first", ctypes.c_float), ("loss_last", ctypes.c_float),
                ("data_ms", ctypes.c_float), ("train_ms", ctypes.c_float)]


class DriftCfg(ctypes.Structure):
    _fields_ = [("theta_mv", ctypes.c_float), ("v_max", ctypes.c_float),
                ("sample_every", ctypes.c_int32), ("hold_steps", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("z_max", ctypes.c_float), ("ca_max", ctypes.c_float)]


class DriftReport(ctypes.Structure):
    _fields_ = [("plain_cell_macro_steps", ctypes.c_int64), ("checked", ctypes.c_int64),
                ("flagged", ctypes.c_int64), ("guarded", ctypes.c_int64), ("ms", ctypes.c_float)]


_lib = None


def lib():
    """Load libinfoli.so; raise when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.infoli_default_options.argtypes = [ctypes.POINTER(Options)]
    L.infoli_default_params.argtypes = [_PF]
    L.infoli_rest_state.argtypes = [_PF, ctypes.c_float, _PF]
    L.infoli_init.argtypes = [ctypes.POINTER(NetworkSpec), ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.infoli_batch_init.argtypes = [ctypes.POINTER(NetworkSpec), ctypes.c_int32,
                                    ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.infoli_step.argtypes = [vp, ctypes.c_int64]
    L.infoli_sync.argtypes = [vp]
    L.infoli_read_state.argtypes = [vp, ctypes.c_int32, _PF, ctypes.c_int64, _PI64]
    L.infoli_read_state_device.argtypes = [vp, ctypes.c_int32, vp]
    L.infoli_write_state.argtypes = [vp, ctypes.c_int32, _PF, ctypes.c_int64]
    L.infoli_read_gap_current.argtypes = [vp, ctypes.c_int32, _PF, ctypes.c_int64]
    L.infoli_read_spikes.argtypes = [vp, ctypes.c_int32, _PI32, ctypes.c_int64, _PF, ctypes.c_int64]
    L.infoli_clear_spikes.argtypes = [vp]
    L.infoli_output_copy_async.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, vp, ctypes.c_int64]
    L.infoli_output_wait.argtypes = [vp]
    L.infoli_get_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.infoli_get_gap_path.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]
    L.infoli_last_step_ms.argtypes = [vp, _PF]
    L.infoli_state_var_name.argtypes = [ctypes.c_int32]
    L.infoli_state_var_name.restype = ctypes.c_char_p
    L.infoli_last_error.argtypes = [vp]
    L.infoli_last_error.restype = ctypes.c_char_p
    L.infoli_destroy.argtypes = [vp]
    L.infoli_destroy.restype = None
    L.infoli_default_train_cfg.argtypes = [ctypes.POINTER(TrainCfg)]
    L.infoli_default_drift_cfg.argtypes = [ctypes.POINTER(DriftCfg)]
    L.infoli_surrogate_train.argtypes = [vp, ctypes.POINTER(TrainCfg), ctypes.POINTER(TrainReport), _PF]
    L.infoli_surrogate_get.argtypes = [vp, _PF, _PF]
    L.infoli_surrogate_set.argtypes = [vp, _PF, _PF]
    L.infoli_step_surrogate.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(DriftCfg),
                                        ctypes.POINTER(DriftReport)]
    L.infoli_mlp_forward.argtypes = [_PF, _PF, ctypes.c_int32, _PF]
    L.infoli_mlp_loss_grad.argtypes = [_PF, _PF, _PF, ctypes.c_int32, _PF, _PF]
    L.infoli_mlp_loss_grad_noalloc.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, vp]
    L.infoli_mlp_adam_step.argtypes = [_PF, _PF, _PF, _PF, ctypes.c_int64, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_float]
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("infoli_state_var_name", "infoli_last_error", "infoli_destroy"):
            fn.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int, ctx=None):
    if status != OK:
        msg = lib().infoli_last_error(ctx).decode()
        raise InfoliError(status, msg)


def _fptr(a):
    return None if a is None else a.ctypes.data_as(_PF)


def default_options(**kw) -> Options:
    o = Options()
    _check(lib().infoli_default_options(ctypes.byref(o)))
    for k, v in kw.items():
        if k == "step_mode" and isinstance(v, str):
            v = MODE[v]
        setattr(o, k, v)
    return o


def default_params() -> np.ndarray:
    p = np.zeros(NUM_PARAMS, np.float32)
    _check(lib().infoli_default_params(_fptr(p)))
    return p


def rest_state(params: Optional[np.ndarray] = None, v0: float = _inputs.REST_MV) -> np.ndarray:
    p = None if params is None else np.ascontiguousarray(params, np.float32)
    out = np.zeros(NUM_STATE, np.float32)
    _check(lib().infoli_rest_state(_fptr(p), ctypes.c_float(v0), _fptr(out)))
    return out


def initial_state(net: "_inputs.Network", v0: float = _inputs.REST_MV) -> np.ndarray:
    """The library's rest state for every cell (each cell's own with
    per-cell parameters) plus the network's jitter."""
    if net.cell_params is None:
        r = rest_state(net.params, v0).astype(np.float64)
        x = np.repeat(r[:, None], net.n, axis=1)
    else:
        x = np.stack([rest_state(net.cell_params[i], v0).astype(np.float64) for i in range(net.n)], axis=1)
    if net.jitter is not None:
        for row, v in enumerate((_inputs.IDX_VD, _inputs.IDX_VS, _inputs.IDX_VA)):
            x[v] += net.jitter[row]
    return np.ascontiguousarray(x.astype(np.float32))


def default_train_cfg(**kw) -> TrainCfg:
    c = TrainCfg()
    _check(lib().infoli_default_train_cfg(ctypes.byref(c)))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def default_drift_cfg(**kw) -> DriftCfg:
    c = DriftCfg()
    _check(lib().infoli_default_drift_cfg(ctypes.byref(c)))
    for k, v in kw.items():
        if k == "mode" and isinstance(v, str):
            v = SURROGATE_MODE[v]
        setattr(c, k, v)
    return c


def _f32(a, n=None):
    a = np.ascontiguousarray(a, np.float32)
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def mlp_forward(params, x) -> np.ndarray:
    """The library's MLP forward kernel on a host batch x [B][16] (B % 16 == 0)."""
    p, xx = _f32(params, MLP_PARAMS), _f32(x)
    y = np.zeros_like(xx)
    _check(lib().infoli_mlp_forward(_fptr(p), _fptr(xx), xx.shape[0], _fptr(y)))
    return y


def mlp_loss_grad(params, x, t):
    """Loss and gradient from the library's forward/backward kernels."""
    p, xx, tt = _f32(params, MLP_PARAMS), _f32(x), _f32(t)
    g = np.zeros(MLP_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    _check(lib().infoli_mlp_loss_grad(_fptr(p), _fptr(xx), _fptr(tt), xx.shape[0], _fptr(loss), _fptr(g)))
    return float(loss[0]), g


def mlp_loss_grad_noalloc(params_ptr: int, x_ptr: int, t_ptr: int, batch: int, loss_ptr: int,
                          grad_ptr: int, stream: int = 0):
    """infoli_mlp_loss_grad_noalloc on device addresses (e.g. a tensor's
    data_ptr()); queued on `stream` (a HIP stream handle, 0 = null stream)."""
    _check(lib().infoli_mlp_loss_grad_noalloc(params_ptr, x_ptr, t_ptr, int(batch), loss_ptr or None,
                                              grad_ptr, stream or None))


def mlp_adam_step(params, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    p, mm, vv = _f32(params, MLP_PARAMS).copy(), _f32(m, MLP_PARAMS).copy(), _f32(v, MLP_PARAMS).copy()
    g = _f32(grad, MLP_PARAMS)
    _check(lib().infoli_mlp_adam_step(_fptr(p), _fptr(mm), _fptr(vv), _fptr(g), int(t), lr, beta1, beta2, eps))
    return p, mm, vv


GAP_KIND = {"rgj": 0, "sgj": 1}
GAP_PATH = ("none", "uniform", "dense", "csr_gather", "csr_chunked", "csr_bitmap", "csr_stream", "uniform_sym",
            "uniform_sum")


class _SpecHolder:
    """Keeps the numpy arrays a NetworkSpec points at alive."""

    def __init__(self, net, init_state=None, i_stream=None, step0=0):
        self.keep = []
        s = NetworkSpec()
        s.n_cells = net.n
        s.dt_ms = net.dt
        s.conn = CONN[net.conn]
        s.g_uniform = float(net.g)
        if net.conn == "dense":
            w = self._f(net.w_dense)
            s.w_dense = _fptr(w)
        if net.conn == "csr":
            rp = np.ascontiguousarray(net.row_ptr, np.int64)
            col = np.ascontiguousarray(net.col, np.int32)
            self.keep += [rp, col]
            s.row_ptr = rp.ctypes.data_as(_PI64)
            s.col = col.ctypes.data_as(_PI32)
            s.nnz = int(rp[-1])
            if net.w_csr is not None:
                s.w_csr = _fptr(self._f(net.w_csr))
        s.params = _fptr(self._f(net.params))
        if init_state is None:
            init_state = initial_state(net)
        s.init_state = _fptr(self._f(init_state))
        if net.bias is not None:
            s.i_bias = _fptr(self._f(net.bias))
        if net.pulses:
            arr = (Pulse * len(net.pulses))()
            for k, p in enumerate(net.pulses):
                arr[k] = Pulse(p.step_begin, p.step_end, p.amplitude, p.cell_begin, p.cell_end)
            self.keep.append(arr)
            s.pulses = arr
            s.n_pulses = len(net.pulses)
        if i_stream is not None:
            st = self._f(i_stream)
            s.i_stream = _fptr(st)
            s.i_stream_steps = st.shape[0]
        s.step0 = step0
        s.gap_kind = GAP_KIND[net.gap]
        if net.cell_params is not None:
            cp = self._f(net.cell_params)
            assert cp.size == net.n * NUM_PARAMS, cp.shape
            s.cell_params = _fptr(cp)
        self.spec = s

    def _f(self, a):
        a = np.ascontiguousarray(a, np.float32)
        self.keep.append(a)
        return a


class Simulator:
    """One library context holding one or more networks."""

    def __init__(self, nets: Union["_inputs.Network", Sequence["_inputs.Network"]],
                 init_states: Optional[List[np.ndarray]] = None,
                 i_streams: Optional[List[np.ndarray]] = None,
                 options: Optional[Options] = None, stream: Optional[int] = None, step0: int = 0,
                 **option_kw):
        self.nets = [nets] if isinstance(nets, _inputs.Network) else list(nets)
        L = lib()
        holders = [_SpecHolder(n, None if init_states is None else init_states[k],
                               None if i_streams is None else i_streams[k], step0)
                   for k, n in enumerate(self.nets)]
        specs = (NetworkSpec * len(holders))(*[h.spec for h in holders])
        opt = options if options is not None else default_options(**option_kw)
        if stream is not None:
            opt.hip_stream = stream
        self.options = opt
        ctx = ctypes.c_void_p()
        _check(L.infoli_batch_init(specs, len(holders), ctypes.byref(opt), ctypes.byref(ctx)))
        self._ctx = ctx
        self.spike_cap = opt.max_spikes_per_cell

    # ----------------------------------------------------------- stepping
    def step(self, n_steps: int):
        _check(lib().infoli_step(self._ctx, int(n_steps)), self._ctx)

    def sync(self):
        _check(lib().infoli_sync(self._ctx), self._ctx)

    def last_step_ms(self) -> float:
        v = ctypes.c_float()
        _check(lib().infoli_last_step_ms(self._ctx, ctypes.byref(v)), self._ctx)
        return float(v.value)

    # ----------------------------------------------------------- state
    def read_state(self, k: int = 0) -> np.ndarray:
        n = self.nets[k].n
        out = np.zeros((NUM_STATE, n), np.float32)
        st = ctypes.c_int64()
        _check(lib().infoli_read_state(self._ctx, k, _fptr(out), out.size, ctypes.byref(st)), self._ctx)
        self.last_step_index = st.value
        return out

    def read_state_device(self, k: int, dev_ptr: int):
        _check(lib().infoli_read_state_device(self._ctx, k, ctypes.c_void_p(dev_ptr)), self._ctx)

    def write_state(self, k: int, x: np.ndarray, step: int):
        x = np.ascontiguousarray(x, np.float32)
        _check(lib().infoli_write_state(self._ctx, k, _fptr(x), int(step)), self._ctx)

    def read_gap_current(self, k: int = 0) -> np.ndarray:
        out = np.zeros(self.nets[k].n, np.float32)
        _check(lib().infoli_read_gap_current(self._ctx, k, _fptr(out), out.size), self._ctx)
        return out

    def read_spikes(self, k: int = 0):
        n = self.nets[k].n
        counts = np.zeros(n, np.int32)
        cap = max(self.spike_cap, 0)
        times = np.zeros((n, cap), np.float32) if cap else None
        _check(lib().infoli_read_spikes(self._ctx, k, counts.ctypes.data_as(_PI32), n,
                                        _fptr(times), 0 if times is None else times.size), self._ctx)
        return counts, times

    # ----------------------------------------------------------- output streaming
    def output_copy_async(self, step_begin: int, n_steps: int, host_ptr: int, cap_floats: int):
        """Queue the copy of the axon voltages after steps [step_begin,
        step_begin + n_steps) into host memory at host_ptr ([n_steps][total
        cells] fp32; pinned memory for overlap); needs output_ring_steps."""
        _check(lib().infoli_output_copy_async(self._ctx, int(step_begin), int(n_steps),
                                              ctypes.c_void_p(host_ptr), int(cap_floats)), self._ctx)

    def output_wait(self):
        _check(lib().infoli_output_wait(self._ctx), self._ctx)

    def clear_spikes(self):
        _check(lib().infoli_clear_spikes(self._ctx), self._ctx)

    def info(self) -> dict:
        i = Info()
        _check(lib().infoli_get_info(self._ctx, ctypes.byref(i)), self._ctx)
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def gap_path(self, k: int = 0):
        """(path name, Vd staged by column blocks) of network k: the form
        its coupling is read in each step."""
        p, blk = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().infoli_get_gap_path(self._ctx, k, ctypes.byref(p), ctypes.byref(blk)), self._ctx)
        return GAP_PATH[p.value], bool(blk.value)

    # ----------------------------------------------------------- surrogate
    def surrogate_train(self, init_params, cfg: Optional[TrainCfg] = None, **kw):
        """Train the MLP surrogate on device-generated transitions; returns
        (report dict, per-step loss array)."""
        c = cfg if cfg is not None else default_train_cfg(**kw)
        p = _f32(init_params, MLP_PARAMS)
        c.init_params = _fptr(p)
        rep = TrainReport()
        hist = np.zeros(max(c.steps, 1), np.float32)
        _check(lib().infoli_surrogate_train(self._ctx, ctypes.byref(c), ctypes.byref(rep), _fptr(hist)),
               self._ctx)
        return {f: getattr(rep, f) for f, _ in TrainReport._fields_}, hist[:c.steps]

    def surrogate_get(self):
        p = np.zeros(MLP_PARAMS, np.float32)
        n = np.zeros(64, np.float32)
        _check(lib().infoli_surrogate_get(self._ctx, _fptr(p), _fptr(n)), self._ctx)
        return p, n

    def surrogate_set(self, params, norm):
        p, n = _f32(params, MLP_PARAMS), _f32(norm, 64)
        _check(lib().infoli_surrogate_set(self._ctx, _fptr(p), _fptr(n)), self._ctx)

    def step_surrogate(self, n_macro: int, cfg: Optional[DriftCfg] = None, report: bool = True, **kw):
        c = cfg if cfg is not None else default_drift_cfg(**kw)
        rep = DriftReport()
        _check(lib().infoli_step_surrogate(self._ctx, int(n_macro), ctypes.byref(c),
                                           ctypes.byref(rep) if report else None), self._ctx)
        return {f: getattr(rep, f) for f, _ in DriftReport._fields_} if report else None

    def close(self):
        if getattr(self, "_ctx", None):
            lib().infoli_destroy(self._ctx)
            self._ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
