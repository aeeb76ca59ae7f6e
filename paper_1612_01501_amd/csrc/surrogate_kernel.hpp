// Surrogate macro step (four time steps of dt) and its training data.
//
// A macro step holds each cell's gap current (computed exactly, in fp32, from
// the Vd at the macro step's start) and evoked input for its four steps; the
// MLP maps the normalised [state, I_gap, I_app] to the normalised state
// increment. The plain method stays the reference and the fallback: cells
// outside the MLP's regime (a voltage above v_max or [Ca] above ca_max), cells
// whose MLP candidate leaves it, cells flagged by an earlier drift check, and
// a rotating sample of cells re-checked this macro step are listed and
// advanced by four plain forward-Euler steps; a checked cell whose MLP result
// differs from the plain one by more than theta in any voltage is flagged for
// a number of macro steps. Every cell advanced by the plain method takes the
// plain result.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cell_model.hpp"
#include "mlp_kernel.hpp"
#include "step_kernel.hpp"

namespace infoli {

// Normalisation: 16 input features (14 states, I_gap, I_app) and 16 outputs
// (14 state increments over the macro step, two pads).
struct NormStats {
    float in_mean[16], in_rstd[16];
    float out_mean[16], out_std[16];
};

struct SurrArgs {
    const float* params;        // fp32 masters (biases)
    const uint16_t* wb;         // bf16 weights
    NormStats norm;
    const float* igap;          // [cells] held gap currents
    int32_t* hold;              // [cells] macro steps left on the plain method
    unsigned long long* counters;   // [0] cells on plain, [1] checked, [2] flagged, [3] guarded
    float theta_mv;             // drift threshold on Vd, Vs, Va
    float v_max;                // regime served by the MLP: every voltage <= v_max
    float ca_max;               //   and [Ca] <= ca_max
    float z_max;                // normalised inputs beyond +-z_max: plain method (0: no bound)
    int32_t sample_every;       // check cells with (cell + macro) % sample_every == 0; 0 = never
    int32_t hold_steps;         // macro steps a flagged cell stays on the plain method
    int32_t mode;               // 0 surrogate, 1 plain for every cell (gap held 4 steps)
    int64_t macro_index;
    struct PlainEntry* list;    // cells for the plain method this macro step: the checked cells
                                // first (cell check_first + i * sample_every at slot i), then
                                // the others, appended
    unsigned int* list_count;   // appended entries; zeroed by the macro step's gap launch
    int64_t check_first;        // first checked cell of this macro step
    int64_t n_checks;           // checked cells (0 when sample_every == 0)
};

// A cell handed to the plain method, with the MLP's candidate voltages (used
// when the cell is checked).
struct PlainEntry {
    int32_t cell;
    float vd, vs, va;
};

// Largest |V| (mV) accepted from the MLP; beyond it the candidate is rejected.
constexpr float kMlpVoltageBound = 150.0f;
// Lanes l, l+16, l+32, l+48 of a wave hold the four feature groups of one cell.
constexpr unsigned long long kCellLanes = 0x0001000100010001ull;

constexpr int kMacro = 4;

// One wave = 16 cells; four lanes per cell (feature groups of four).
static __global__ __launch_bounds__(256) void k_surrogate_step(StepArgs a, SurrArgs s, const float* __restrict__ xin,
                                                        float* __restrict__ xout, int64_t step0,
                                                        int64_t n_cells_total) {
    __shared__ __align__(16) uint16_t s_w[kMlpLdsElems];
    const MlpSmem sm = mlp_smem(s_w);
    if (s.mode == 0) {
        load_weights_lds(s.wb, sm);
        __syncthreads();
    }
    const int l = threadIdx.x & 63;
    const int g = l >> 4;
    const int waves = blockDim.x >> 6;
    for (int64_t base = ((int64_t)blockIdx.x * waves + (threadIdx.x >> 6)) * 16; base < n_cells_total;
         base += (int64_t)gridDim.x * waves * 16) {
        const int64_t cell = base + (l & 15);
        const bool live = cell < n_cells_total;
        const int64_t c = live ? cell : n_cells_total - 1;
        const InstDesc& d = a.inst[0];      // surrogate contexts hold one network
        const int li = (int)(c - d.cell_off);
        const float ig = s.igap[c];
        const float ia0 = evoked_input(a, d, step0, li, c);

        // reasons known before the MLP runs (the same on the cell's four lanes)
        const float vd0 = xin[SV_VD * a.stride + c];
        const float vs0 = xin[SV_VS * a.stride + c];
        const float va0 = xin[SV_VA * a.stride + c];
        const float ca0 = xin[SV_CA * a.stride + c];
        const bool in_regime = fmaxf(vd0, fmaxf(vs0, va0)) <= s.v_max && ca0 <= s.ca_max;
        const int hold = s.hold[c];
        const bool check = s.sample_every > 0 &&
                           ((c + s.macro_index) % s.sample_every) == 0;

        // MLP on every lane (the matrix cores need the whole wave)
        f32x4 y = {0.0f, 0.0f, 0.0f, 0.0f};
        f32x4 xg;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int v = 4 * g + e;
            xg[e] = v < NSV ? xin[v * a.stride + c] : 0.0f;
        }
        bool far = false;       // a normalised input of this lane's group outside the bound
        if (s.mode == 0) {
            f32x4 xnv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int v = 4 * g + e;
                const float raw = v < NSV ? xg[e] : (v == 14 ? ig : ia0);
                xnv[e] = (raw - s.norm.in_mean[v]) * s.norm.in_rstd[v];
                far = far || !(fabsf(xnv[e]) <= s.z_max);
            }
            if (!(s.z_max > 0.0f)) far = false;
            y = mlp_forward(sm, s.params, pack_bf16(xnv), nullptr, nullptr);
        }
        const bool cell_far = ((__ballot(far) >> (l & 15)) & kCellLanes) != 0;
        // MLP candidate: x + denormalised increment (lane holds 4 variables)
        f32x4 xm;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int v = 4 * g + e;
            xm[e] = xg[e] + (y[e] * s.norm.out_std[v] + s.norm.out_mean[v]);
        }
        // voltages of the MLP candidate, gathered to the cell's group-0 lane
        const float mvd = __shfl(xm[0], (l & 15), 64);           // v = 0  (g 0, e 0)
        const float mvs = __shfl(xm[1], (l & 15) + 16, 64);      // v = 5  (g 1, e 1)
        const float mva = __shfl(xm[3], (l & 15) + 32, 64);      // v = 11 (g 2, e 3)

        // Guards, tested every macro step: a cell outside the regime the MLP
        // was trained on, with inputs far from the training data, or whose
        // MLP candidate leaves the regime (or is unusable) takes the plain
        // method for this macro step.
        const bool cand_bad = !(fabsf(mvd) <= kMlpVoltageBound && fabsf(mvs) <= kMlpVoltageBound &&
                                fabsf(mva) <= kMlpVoltageBound) ||
                              fmaxf(mvd, fmaxf(mvs, mva)) > s.v_max;
        const bool guard = s.mode == 0 && (!in_regime || cell_far || cand_bad);
        const bool plain = s.mode == 1 || hold > 0 || check || guard;

        // guarded cells counted with one atomic per wave that has any
        const bool lead = g == 0 && live;
        const unsigned long long n_guard = __popcll(__ballot(lead && guard));

        if (!plain) {
            if (live)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int v = 4 * g + e;
                    if (v < NSV) xout[v * a.stride + c] = xm[e];
                }
            // spike of an MLP cell: Va crossing 0 mV within the macro step
            if (g == 0 && live) {
                if (va0 < 0.0f && mva >= 0.0f) {
                    const int cnt = a.spike_count[c];
                    if (a.spike_cap > 0) {
                        const float frac = (0.0f - va0) / (mva - va0);
                        a.spike_times[c * a.spike_cap + (cnt % a.spike_cap)] =
                            ((float)step0 + kMacro * frac) * a.dt;
                    }
                    a.spike_count[c] = cnt + 1;
                }
            }
        }
        // cells for the plain method: a checked cell at its own slot (no
        // atomic); the others appended after the checked ones, one atomic per
        // wave that has any
        if (lead && plain && check)
            s.list[(int32_t)(c - s.check_first) / s.sample_every] = PlainEntry{(int32_t)c, mvd, mvs, mva};
        const unsigned long long pmask = __ballot(lead && plain && !check);
        if (pmask) {
            unsigned int base = 0;
            if (l == 0) base = atomicAdd(s.list_count, (unsigned int)__popcll(pmask));
            base = __shfl(base, 0, 64);
            if (lead && plain && !check) {
                const unsigned int pos = base + (unsigned int)__popcll(pmask & ((1ull << l) - 1ull));
                s.list[s.n_checks + pos] = PlainEntry{(int32_t)c, mvd, mvs, mva};
            }
        }
        if (l == 0 && n_guard) atomicAdd(&s.counters[3], n_guard);
    }
}

// The listed cells: four plain forward-Euler steps with the macro step's gap
// current held, spike detection, and for checked cells the drift test
// against the MLP candidate (past theta: hold_steps macro steps of plain
// method). A workgroup of two waves takes 64 listed cells: wave 0 advances
// their dendrite and axon, wave 1 their soma (cell_step's arithmetic, split
// by compartment); the state is exchanged through LDS after every step.
constexpr int kListBlock = 128;

static __global__ __launch_bounds__(kListBlock) void k_plain_list(StepArgs a, SurrArgs s,
                                                                  const float* __restrict__ xin,
                                                                  float* __restrict__ xout, int64_t step0) {
    __shared__ float s_x[2][NSV][64];
    const int64_t count = s.n_checks + *s.list_count;   // checked cells first, then the appended
    const InstDesc& d = a.inst[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        atomicAdd(&s.counters[0], (unsigned long long)count);
        if (s.n_checks) atomicAdd(&s.counters[1], (unsigned long long)s.n_checks);
    }
    const int lane = threadIdx.x & 63;
    const int part = threadIdx.x >> 6;        // 0: dendrite and axon, 1: soma
    for (int64_t b = (int64_t)blockIdx.x * 64; b < count; b += (int64_t)gridDim.x * 64) {
        const int64_t i = b + lane;
        const bool act = i < count;
        PlainEntry e{0, 0.0f, 0.0f, 0.0f};
        if (act) e = s.list[i];
        const int64_t c = e.cell;            // cell 0 for idle lanes: read, never written
        const int li = (int)(c - d.cell_off);
        const float ig = s.igap[c];
        float x[NSV], y[NSV];
#pragma unroll
        for (int v = 0; v < NSV; ++v) x[v] = xin[v * a.stride + c];
        int cnt = part == 0 ? a.spike_count[c] : 0;
        for (int k = 0; k < kMacro; ++k) {
            const int64_t st = step0 + k;
            if (part == 0) {
                cell_step_dendrite(d.p, x, ig, evoked_input(a, d, st, li, c), a.dt, y);
                cell_step_axon(d.p, x, a.dt, y);
                if (x[SV_VA] < 0.0f && y[SV_VA] >= 0.0f) {
                    if (act && a.spike_cap > 0) {
                        const float frac = (0.0f - x[SV_VA]) / (y[SV_VA] - x[SV_VA]);
                        a.spike_times[c * a.spike_cap + (cnt % a.spike_cap)] = ((float)st + frac) * a.dt;
                    }
                    ++cnt;
                }
#pragma unroll
                for (int v : {SV_VD, SV_CA, SV_R, SV_S, SV_Q, SV_VA, SV_HA, SV_XA}) s_x[k & 1][v][lane] = y[v];
            } else {
                cell_step_soma(d.p, x, a.dt, y);
#pragma unroll
                for (int v : {SV_VS, SV_K, SV_L, SV_H, SV_N, SV_X}) s_x[k & 1][v][lane] = y[v];
            }
            // one barrier per step: buffer k & 1 is rewritten two steps later,
            // after every thread has passed the next barrier
            __syncthreads();
#pragma unroll
            for (int v = 0; v < NSV; ++v) x[v] = s_x[k & 1][v][lane];
        }
        bool flagged = false;
        if (act) {
            float chk = 0.0f;
            if (part == 0) {
                a.spike_count[c] = cnt;
#pragma unroll
                for (int v : {SV_VD, SV_CA, SV_R, SV_S, SV_Q, SV_VA, SV_HA, SV_XA}) {
                    xout[v * a.stride + c] = x[v];
                    chk += x[v];
                }
            } else {
#pragma unroll
                for (int v : {SV_VS, SV_K, SV_L, SV_H, SV_N, SV_X}) {
                    xout[v * a.stride + c] = x[v];
                    chk += x[v];
                }
            }
            if (!isfinite(chk)) atomicOr(a.flags, 1);
            if (part == 0) {
                const int hold = s.hold[c];
                int new_hold = hold > 0 ? hold - 1 : 0;
                if (i < s.n_checks) {
                    const float dev =
                        fmaxf(fabsf(e.vd - x[SV_VD]), fmaxf(fabsf(e.vs - x[SV_VS]), fabsf(e.va - x[SV_VA])));
                    if (!(dev <= s.theta_mv)) {
                        new_hold = s.hold_steps;
                        flagged = true;
                    }
                }
                if (new_hold != hold) s.hold[c] = new_hold;
            }
        }
        const unsigned long long fm = __ballot(flagged);
        if (lane == 0 && fm) atomicAdd(&s.counters[2], (unsigned long long)__popcll(fm));
    }
}

// Four plain forward-Euler steps per cell with the macro step's gap current
// held (the surrogate's ablation without the MLP): one thread per cell.
static __global__ __launch_bounds__(256) void k_hold4(StepArgs a, const float* __restrict__ igap,
                                                      const float* __restrict__ xin, float* __restrict__ xout,
                                                      int64_t step0, int64_t n_cells_total) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells_total) return;
    const InstDesc& d = a.inst[0];
    const int li = (int)(c - d.cell_off);
    const float ig = igap[c];
    float x[NSV], y[NSV];
#pragma unroll
    for (int v = 0; v < NSV; ++v) x[v] = xin[v * a.stride + c];
    int cnt = a.spike_count[c];
    const int cnt0 = cnt;
    for (int k = 0; k < kMacro; ++k) {
        const int64_t st = step0 + k;
        cell_step(d.p, x, ig, evoked_input(a, d, st, li, c), a.dt, y);
        if (x[SV_VA] < 0.0f && y[SV_VA] >= 0.0f) {
            if (a.spike_cap > 0) {
                const float frac = (0.0f - x[SV_VA]) / (y[SV_VA] - x[SV_VA]);
                a.spike_times[c * a.spike_cap + (cnt % a.spike_cap)] = ((float)st + frac) * a.dt;
            }
            ++cnt;
        }
#pragma unroll
        for (int v = 0; v < NSV; ++v) x[v] = y[v];
    }
    if (cnt != cnt0) a.spike_count[c] = cnt;
    float chk = 0.0f;
#pragma unroll
    for (int v = 0; v < NSV; ++v) {
        xout[v * a.stride + c] = x[v];
        chk += x[v];
    }
    if (!isfinite(chk)) atomicOr(a.flags, 1);
}

// ---------------------------------------------------------------- training data
// Independent cells driven by random currents, advanced by the plain method:
// each macro step records (state, I_gap, I_app) and the state increment over
// four steps with both currents held. Only transitions the surrogate would be
// asked to make are recorded: those starting in its regime (every voltage
// <= v_max, [Ca] <= ca_max); the trajectory itself runs on through spikes. A
// trajectory that records nothing for kMaxIdle macro steps, or leaves the
// model's range, restarts from the (jittered) rest state. Per trajectory: a constant bias
// N(0, bias_sd); a gap current following an AR(1) process with stationary
// standard deviation gap_sd and lag-one correlation gap_rho per macro step;
// pulses of amplitude U[pulse_lo, pulse_hi] lasting pulse_len macro steps,
// starting with probability pulse_p per macro step; a burn-in drawn uniformly
// from [0, burn_in] macro steps before recording. Initial state: rest plus
// U[-1, 1] mV on the three voltages. Random numbers: SplitMix64 finaliser of
// (seed, trajectory, macro step, stream), uniform in (0, 1) from 24 bits.
struct DataGenArgs {
    CellParams p;
    float rest[NSV];
    float dt;
    float bias_sd, gap_sd, gap_rho, pulse_p, pulse_lo, pulse_hi;
    float v_max, ca_max;      // regime: transitions starting outside are not recorded
    int32_t pulse_len;
    int32_t burn_in;          // largest number of unrecorded macro steps
    int32_t per_traj;         // recorded macro steps per trajectory
    int32_t n_traj;
    uint64_t seed;
    float* x_raw;             // [N][16] state, I_gap, I_app
    float* d_raw;             // [N][16] increments (pads zero)
};

__device__ __forceinline__ float u01(uint64_t seed, uint64_t traj, uint64_t m, uint64_t stream) {
    const uint64_t h = mix64(seed ^ mix64(traj * 0x100000001b3ull + (m << 8) + stream));
    return ((float)(h >> 40) + 0.5f) * (1.0f / 16777216.0f);
}
__device__ __forceinline__ float normal01(uint64_t seed, uint64_t traj, uint64_t m, uint64_t stream) {
    // Box-Muller
    const float u1 = u01(seed, traj, m, stream), u2 = u01(seed, traj, m, stream + 1);
    return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

constexpr int kMaxIdle = 4000;

__device__ __forceinline__ void rest_jittered(const DataGenArgs& g, uint64_t t, uint64_t m, float* x) {
#pragma unroll
    for (int v = 0; v < NSV; ++v) x[v] = g.rest[v];
    x[SV_VD] += 2.0f * u01(g.seed, t, m, 10) - 1.0f;
    x[SV_VS] += 2.0f * u01(g.seed, t, m, 11) - 1.0f;
    x[SV_VA] += 2.0f * u01(g.seed, t, m, 12) - 1.0f;
}

// Termination: after the burn-in every macro step either records or counts
// towards kMaxIdle; a restart puts the voltages at -60 +- 1 mV and [Ca] at
// rest, inside the regime (the host requires v_max >= -50 mV and ca_max above
// the rest value), so the next step records.
static __global__ void k_surrogate_data(DataGenArgs g) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.n_traj) return;
    float x[NSV], y[NSV];
    rest_jittered(g, t, 0, x);
    const float bias = g.bias_sd * normal01(g.seed, t, 0, 20);
    float gap = g.gap_sd * normal01(g.seed, t, 0, 30);
    int pulse_left = 0;
    float pulse_amp = 0.0f;
    const float innov = g.gap_sd * sqrtf(1.0f - g.gap_rho * g.gap_rho);
    // burn-in of this trajectory: uniform in [0, burn_in] macro steps, so the
    // recorded states cover the slow variables' whole excursion
    const int burn = (int)(u01(g.seed, t, 0, 60) * (float)(g.burn_in + 1));
    int idle = 0, rec = 0;
    for (int64_t m = 1; rec < g.per_traj; ++m) {
        if (idle > kMaxIdle) {
            rest_jittered(g, t, m, x);
            gap = 0.0f;
            pulse_left = 0;
            idle = 0;
        }
        gap = g.gap_rho * gap + innov * normal01(g.seed, t, m, 40);
        if (pulse_left == 0 && u01(g.seed, t, m, 50) < g.pulse_p) {
            pulse_left = g.pulse_len;
            pulse_amp = g.pulse_lo + (g.pulse_hi - g.pulse_lo) * u01(g.seed, t, m, 51);
        }
        float iapp = bias + (pulse_left > 0 ? pulse_amp : 0.0f);
        if (pulse_left > 0) --pulse_left;
        float x0[NSV];
#pragma unroll
        for (int v = 0; v < NSV; ++v) x0[v] = x[v];
        bool served = fmaxf(x0[SV_VD], fmaxf(x0[SV_VS], x0[SV_VA])) <= g.v_max && x0[SV_CA] <= g.ca_max;
        for (int k = 0; k < kMacro; ++k) {
            cell_step(g.p, x, gap, iapp, g.dt, y);
#pragma unroll
            for (int v = 0; v < NSV; ++v) x[v] = y[v];
        }
        // a trajectory driven out of the model's range (forward Euler loses
        // stability for very large currents) restarts from the rest state
        float chk = 0.0f;
#pragma unroll
        for (int v = 0; v < NSV; ++v) chk += x[v];
        if (!isfinite(chk) || fabsf(x[SV_VD]) > 150.0f || fabsf(x[SV_VS]) > 150.0f || fabsf(x[SV_VA]) > 150.0f) {
#pragma unroll
            for (int v = 0; v < NSV; ++v) x[v] = x0[v] = g.rest[v];
            gap = 0.0f;
            pulse_left = 0;
            iapp = bias;
            served = true;
            for (int k = 0; k < kMacro; ++k) {
                cell_step(g.p, x, gap, bias, g.dt, y);
#pragma unroll
                for (int v = 0; v < NSV; ++v) x[v] = y[v];
            }
        }
        if (m <= burn) continue;
        if (!served) {
            ++idle;
            continue;
        }
        idle = 0;
        const int64_t r = (int64_t)rec * g.n_traj + t;
        ++rec;
        float* xr = g.x_raw + r * 16;
        float* dr = g.d_raw + r * 16;
#pragma unroll
        for (int v = 0; v < NSV; ++v) {
            xr[v] = x0[v];
            dr[v] = x[v] - x0[v];
        }
        xr[14] = gap;
        xr[15] = iapp;
        dr[14] = 0.0f;
        dr[15] = 0.0f;
    }
}

// Per-feature mean and standard deviation of a [N][16] array: one workgroup
// per feature, fixed-order fp64 reduction.
static __global__ __launch_bounds__(256) void k_feature_stats(const float* __restrict__ a, int64_t n,
                                                       double* __restrict__ out /* [16][2] */) {
    __shared__ double s1[256], s2[256];
    const int f = blockIdx.x;
    double m = 0.0, q = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const double v = a[r * 16 + f];
        m += v;
        q += v * v;
    }
    s1[threadIdx.x] = m;
    s2[threadIdx.x] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = s1[0] / (double)n;
        const double var = s2[0] / (double)n - mean * mean;
        out[2 * f] = mean;
        out[2 * f + 1] = var > 0.0 ? sqrt(var) : 0.0;
    }
}

// In-place normalisation of inputs and targets.
static __global__ void k_normalize(float* __restrict__ x, float* __restrict__ t, int64_t n, NormStats ns) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * 16) return;
    const int f = (int)(e % 16);
    x[e] = (x[e] - ns.in_mean[f]) * ns.in_rstd[f];
    t[e] = f < kTargets ? (t[e] - ns.out_mean[f]) / ns.out_std[f] : 0.0f;
}

}  // namespace infoli
