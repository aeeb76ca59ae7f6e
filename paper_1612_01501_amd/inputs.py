"""Seeded synthetic inputs for the InfOli workloads.

This module is shared by the GPU library's callers (tests, benchmark) and by
the CPU oracle's tests. It holds input data and random draws only, none of
the simulation arithmetic: the per-cell conductance table (the 20 "neuron
conductances" of the paper's Table 1, given as data), voltage jitter, input
biases, pulse lists and random gap-junction graphs.

Workload shapes follow the paper's networks (Section 3: 96-7,680 cells,
connectivity densities 0-100 %) and the configurations the library is
measured on; every draw takes an explicit seed.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

# Order of the 20 per-cell parameters (conductances in mS/cm^2, area ratios,
# reversal potentials in mV).
PARAM_NAMES = (
    "g_CaH", "g_KCa", "g_h", "g_ld", "g_CaL", "g_Na_s", "g_Kdr_s", "g_K_s",
    "g_ls", "g_Na_a", "g_K_a", "g_la", "g_int", "p1", "p2",
    "V_Na", "V_K", "V_Ca", "V_h", "V_L",
)

# Default values of the published three-compartment inferior-olive cell
# (De Gruijl et al., PLoS Comput Biol 8, 2012; dendrite/soma channels from
# Schweighofer et al., J Neurophysiol 82, 1999).
DEFAULT_PARAMS = np.array([
    4.5,     # g_CaH   dendritic high-threshold Ca
    35.0,    # g_KCa   dendritic Ca-activated K
    0.125,   # g_h     dendritic h current
    0.016,   # g_ld    dendritic leak
    0.68,    # g_CaL   somatic low-threshold Ca
    150.0,   # g_Na_s  somatic Na
    9.0,     # g_Kdr_s somatic delayed-rectifier K
    5.0,     # g_K_s   somatic K
    0.016,   # g_ls    somatic leak
    240.0,   # g_Na_a  axonal Na
    20.0,    # g_K_a   axonal K
    0.016,   # g_la    axonal leak
    0.13,    # g_int   internal (inter-compartment) conductance
    0.25,    # p1      soma/dendrite area ratio
    0.15,    # p2      axon/soma area ratio
    55.0,    # V_Na
    -75.0,   # V_K
    120.0,   # V_Ca
    -43.0,   # V_h
    10.0,    # V_L
], dtype=np.float64)

STATE_NAMES = ("Vd", "Ca", "r", "s", "q", "Vs", "k", "l", "h", "n", "x",
               "Va", "ha", "xa")
N_STATE = len(STATE_NAMES)
IDX_VD, IDX_VS, IDX_VA = 0, 5, 11

DT_MS = 0.05          # Section 2.2: 50 us per step
REST_MV = -60.0       # voltage of the rest state


@dataclasses.dataclass
class Pulse:
    step_begin: int     # active for integer steps step_begin <= n < step_end
    step_end: int
    amplitude: float    # uA/cm^2
    cell_begin: int = 0
    cell_end: int = -1  # -1 => every cell


@dataclasses.dataclass
class Network:
    """One network instance, host arrays only."""
    n: int
    conn: str                       # "none" | "uniform" | "dense" | "csr"
    g: float = 0.0                  # uniform conductance, mS/cm^2
    w_dense: Optional[np.ndarray] = None   # [n, n] float32, row i = into i
    row_ptr: Optional[np.ndarray] = None   # [n+1] int64
    col: Optional[np.ndarray] = None       # [nnz] int32
    w_csr: Optional[np.ndarray] = None     # [nnz] float32 or None => g
    jitter: Optional[np.ndarray] = None    # [3, n] mV offsets on Vd, Vs, Va
    bias: Optional[np.ndarray] = None      # [n] float32, uA/cm^2
    pulses: List[Pulse] = dataclasses.field(default_factory=list)
    params: np.ndarray = dataclasses.field(default_factory=lambda: DEFAULT_PARAMS.copy())
    dt: float = DT_MS
    gap: str = "rgj"                # "rgj": realistic gap junctions | "sgj": simplified (linear)
    cell_params: Optional[np.ndarray] = None  # [n, 20]: per-cell values, else params for every cell
    label: str = ""

    @property
    def nnz(self) -> int:
        if self.conn == "csr":
            return int(self.row_ptr[-1])
        if self.conn in ("uniform", "dense"):
            return self.n * (self.n - 1) if self.conn == "uniform" else self.n * self.n
        return 0

    def pairs_per_step(self) -> int:
        """Directed gap pair-interactions that contribute per step."""
        if self.conn == "uniform":
            return self.n * (self.n - 1)
        if self.conn == "dense":
            return int(np.count_nonzero(self.w_dense))
        if self.conn == "csr":
            return int(self.row_ptr[-1])
        return 0


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def voltage_jitter(n: int, seed: int, amplitude_mv: float = 1.0) -> np.ndarray:
    """Independent U[-a, +a] mV offsets for Vd, Vs and Va of every cell."""
    return rng(seed).uniform(-amplitude_mv, amplitude_mv, size=(3, n))


def input_bias(n: int, seed: int, sigma: float = 0.5) -> np.ndarray:
    """Constant per-cell input current drawn once from N(0, sigma^2)."""
    return rng(seed).normal(0.0, sigma, size=n).astype(np.float32)


def erdos_renyi_csr(n: int, p: float, seed: int):
    """Symmetric Erdos-Renyi graph without self-loops as sorted CSR.

    Every unordered pair i < j is present independently with probability p;
    a present pair adds the directed edges (i, j) and (j, i). Networks above
    16,384 cells draw the present pairs by geometric skips over the upper
    triangle instead of one uniform per pair (same distribution).
    """
    if n > 16384 and 0.0 < p < 1.0:
        return _erdos_renyi_skip(n, p, seed)
    g = rng(seed)
    rows, cols = [], []
    block = max(1, int(4_000_000 // max(n, 1)))
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        u = g.random((i1 - i0, n))
        ii, jj = np.nonzero(u < p)
        ii = ii + i0
        keep = jj > ii
        rows.append(ii[keep])
        cols.append(jj[keep])
    r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    src = np.concatenate([r, c])
    dst = np.concatenate([c, r])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, dst.astype(np.int32)


def _erdos_renyi_skip(n: int, p: float, seed: int):
    g = rng(seed)
    total = n * (n - 1) // 2                      # pairs i < j, row-major over i
    chunks, pos = [], -1
    while True:
        k = int(max(1024, (total - pos) * p * 1.05 + 10 * np.sqrt(total * p) + 1024))
        gaps = g.geometric(p, size=k).astype(np.int64)
        loc = pos + np.cumsum(gaps)
        inside = loc[loc < total]
        chunks.append(inside)
        if len(inside) < len(loc):
            break
        pos = int(loc[-1])
    t = np.concatenate(chunks)
    # pair index -> (i, j): t = i*(2n-i-1)/2 + (j - i - 1)
    i = (n - 2 - np.floor(np.sqrt(-8.0 * t + 4.0 * n * (n - 1) - 7.0) / 2.0 - 0.5)).astype(np.int64)
    first = i * (2 * n - i - 1) // 2
    i = np.where(first > t, i - 1, i)
    first = i * (2 * n - i - 1) // 2
    nxt = (i + 1) * (2 * n - i - 2) // 2
    i = np.where(nxt <= t, i + 1, i)
    first = i * (2 * n - i - 1) // 2
    j = t - first + i + 1
    # forward edges (i, j) are sorted by (i, j); reverse edges (j, i) by (j, i)
    order = np.argsort(j * n + i, kind="stable")
    rr, rc = j[order], i[order]
    cnt_f = np.bincount(i, minlength=n)
    cnt_r = np.bincount(rr, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt_f + cnt_r, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    off_r = np.concatenate([[0], np.cumsum(cnt_r)[:-1]])
    off_f = np.concatenate([[0], np.cumsum(cnt_f)[:-1]])
    col[row_ptr[:-1][rr] + (np.arange(len(rr)) - off_r[rr])] = rc
    col[row_ptr[:-1][i] + cnt_r[i] + (np.arange(len(i)) - off_f[i])] = j
    return row_ptr, col


def complete_csr(n: int):
    """All-to-all graph without self-loops as CSR."""
    row_ptr = np.arange(n + 1, dtype=np.int64) * (n - 1)
    col = np.empty(n * (n - 1), dtype=np.int32)
    base = np.arange(n, dtype=np.int32)
    for i in range(n):
        col[i * (n - 1):(i + 1) * (n - 1)] = np.concatenate([base[:i], base[i + 1:]])
    return row_ptr, col


# ---------------------------------------------------------------- workloads
def config0(seed: int = 0, n: int = 96) -> Network:
    """96 cells all-to-all, g = 0.04, jitter +-1 mV, 6 uA/cm^2 pulse on the
    dendrite during steps [400, 500) (t = 20..25 ms) of a 2,000-step run."""
    return Network(n=n, conn="uniform", g=0.04,
                   jitter=voltage_jitter(n, 2000 + seed),
                   pulses=[Pulse(400, 500, 6.0)], label=f"c0_uniform_n{n}")


def config1(density: float, seed: int = 0, n: int = 4096) -> Network:
    """4,096 cells, symmetric ER graph at the given density stored as CSR with
    g = 0.04 on every edge, per-cell bias N(0, 0.5), pulse as config 0."""
    row_ptr, col = erdos_renyi_csr(n, density, 1000 + seed)
    return Network(n=n, conn="csr", g=0.04, row_ptr=row_ptr, col=col,
                   jitter=voltage_jitter(n, 2000 + seed),
                   bias=input_bias(n, 3000 + seed),
                   pulses=[Pulse(400, 500, 6.0)],
                   label=f"c1_csr_n{n}_p{density:g}")


def config2(seed: int = 0, n: int = 16384, pulse: bool = False) -> Network:
    """16,384 cells dense all-to-all with g = 0.04 * 96 / N and jitter; no
    input (a pulse variant exists for spike checks)."""
    return Network(n=n, conn="uniform", g=0.04 * 96.0 / n,
                   jitter=voltage_jitter(n, 2000 + seed),
                   pulses=[Pulse(400, 500, 6.0)] if pulse else [],
                   label=f"c2_uniform_n{n}")


def config3(seed: int = 0, n_instances: int = 256, n_min: int = 64,
            n_max: int = 2048) -> List[Network]:
    """Uneven batch: N_k ~ U{n_min..n_max}, density ~ U{5 %, 25 %, 100 %},
    g_k ~ U[0.01, 0.08], pulse amplitude A_k ~ U[2, 10] during [400, 500)."""
    g = rng(4000 + seed)
    sizes = g.integers(n_min, n_max + 1, size=n_instances)
    dens = g.choice(np.array([0.05, 0.25, 1.0]), size=n_instances)
    gs = g.uniform(0.01, 0.08, size=n_instances)
    amps = g.uniform(2.0, 10.0, size=n_instances)
    nets = []
    for k in range(n_instances):
        n = int(sizes[k])
        jit = voltage_jitter(n, 2000 + seed * 100003 + k)
        if dens[k] >= 1.0:
            net = Network(n=n, conn="uniform", g=float(gs[k]), jitter=jit)
        else:
            rp, c = erdos_renyi_csr(n, float(dens[k]), 1000 + seed * 100003 + k)
            net = Network(n=n, conn="csr", g=float(gs[k]), row_ptr=rp, col=c, jitter=jit)
        net.pulses = [Pulse(400, 500, float(amps[k]))]
        net.label = f"c3_k{k}_n{n}_p{dens[k]:g}"
        nets.append(net)
    return nets


def config4_graph(seed: int = 0, n: int = 65536, degree: float = 1000.0):
    """Symmetric ER graph of mean degree `degree` for the 65,536-cell network."""
    return erdos_renyi_csr(n, degree / (n - 1), 1000 + seed)


def config4(seed: int = 0, n: int = 65536, degree: float = 1000.0) -> Network:
    row_ptr, col = config4_graph(seed, n, degree)
    return Network(n=n, conn="csr", g=0.04 * 96.0 / 1000.0, row_ptr=row_ptr, col=col,
                   jitter=voltage_jitter(n, 2000 + seed),
                   bias=input_bias(n, 3000 + seed),
                   pulses=[Pulse(400, 500, 6.0)], label=f"c4_csr_n{n}_deg{degree:g}")


# ---------------------------------------------------------------- surrogate MLP
MLP_K_IN, MLP_HID, MLP_K_OUT = 16, 128, 16


def mlp_init_params(seed: int = 5000) -> np.ndarray:
    """Initial MLP parameters (flat fp32, order W1 b1 W2 b2 W3 b3 with
    W1 [128][16], W2 [128][128], W3 [16][128]): weights U(-1/sqrt(fan_in),
    1/sqrt(fan_in)), biases zero."""
    g = rng(seed)
    parts = []
    for rows, cols in ((MLP_HID, MLP_K_IN), (MLP_HID, MLP_HID), (MLP_K_OUT, MLP_HID)):
        b = 1.0 / np.sqrt(cols)
        parts.append(g.uniform(-b, b, rows * cols))
        parts.append(np.zeros(rows))
    return np.concatenate(parts).astype(np.float32)


def mlp_batch(n: int, seed: int):
    """A synthetic training batch: inputs ~ N(0, 1) in R^16, targets ~ N(0, 1)."""
    g = rng(seed)
    return (g.normal(0.0, 1.0, (n, MLP_K_IN)).astype(np.float32),
            g.normal(0.0, 1.0, (n, MLP_K_OUT)).astype(np.float32))
