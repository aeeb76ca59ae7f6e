/*
 * infoli.h - C ABI of the MI355X (gfx950) InfOli network simulator.
 *
 * The library advances networks of three-compartment inferior-olive cells
 * (dendrite, soma, axon) coupled through dendritic gap junctions, the
 * workload of Smaragdos et al., "BrainFrame" (arXiv:1612.01501):
 *
 *   - Section 2.2: every step n -> n+1 updates all compartments of all cells
 *     and all gap junctions from the step-n state only (synchronous forward
 *     Euler, dt = 50 us by default); each cell gets one evoked input value per
 *     step; its output is the axon voltage.
 *   - Section 2.3 (Algorithm 1): the gap current into cell i is
 *       I_gap,i = sum_j w_ij * dV * (0.8 * exp(-dV^2 / 100) + 0.2),
 *       dV = Vd_i - Vd_j  (mV; w in mS/cm^2; I in uA/cm^2),
 *     an outward current of the dendrite. Connectivity is an N x N weight
 *     matrix given before the run (Section 2.3), stored uniform, dense or CSR.
 *   - Section 2.4.3: the whole run's inputs are placed on the device once at
 *     initialisation; no host-to-device traffic happens while stepping.
 *
 * Conventions (all entry points):
 *   - Every function returns an infoli_status; none aborts, exits or lets a
 *     C++ exception escape. On failure nothing observable changes and
 *     infoli_last_error() describes the failure.
 *   - Host pointers are read during the call only: the caller keeps ownership
 *     and may free them when the call returns. Output buffers are allocated
 *     by the caller, with an explicit capacity; a too-small capacity returns
 *     INFOLI_E_INVALID_ARG and writes nothing.
 *   - A context owns all device memory it allocates; infoli_destroy frees it.
 *     A context is used by one host thread at a time; contexts are independent.
 *   - Device work is queued on the context's stream (the caller's HIP stream
 *     when options.hip_stream is set, else a stream the context owns).
 *     infoli_step only queues work; infoli_sync and the read functions wait.
 *   - State is structure-of-arrays, float32: element (v, i) of an instance
 *     with n cells is at offset v * n + i, v in [0, INFOLI_NUM_STATE).
 *   - Results are deterministic: repeated runs give bitwise identical states
 *     (fixed reduction order, no floating-point atomics).
 */
#ifndef INFOLI_API_H_
#define INFOLI_API_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum infoli_status {
    INFOLI_OK = 0,
    INFOLI_E_INVALID_ARG = 1,   /* NULL pointer, bad size, bad enum, capacity too small */
    INFOLI_E_BAD_GRAPH = 2,     /* CSR not monotone, column out of range or a row's columns
                                   not strictly ascending, non-finite weight                 */
    INFOLI_E_OUT_OF_MEMORY = 3, /* device or host allocation failed                        */
    INFOLI_E_DEVICE = 4,        /* HIP runtime error, or no gfx950 device                   */
    INFOLI_E_NUMERIC = 5,       /* a state value became NaN or infinite while stepping      */
    INFOLI_E_STATE = 6,         /* call not valid in the context's current state            */
    INFOLI_E_UNSUPPORTED = 7    /* valid request that the library does not implement       */
} infoli_status;

/* Connectivity storage of one network (Section 2.3: N x N weights). */
typedef enum infoli_conn {
    INFOLI_CONN_NONE = 0,        /* no gap junctions (independent cells)                    */
    INFOLI_CONN_UNIFORM_ALL = 1, /* all-to-all, w_ij = g_uniform for i != j                 */
    INFOLI_CONN_DENSE = 2,       /* explicit n*n row-major matrix, row i = weights INTO i   */
    INFOLI_CONN_CSR = 3          /* CSR by receiving cell: row i lists the j coupled to i   */
} infoli_conn;

/* Form of the gap-junction term of one connection (dV = Vd_i - Vd_j). */
typedef enum infoli_gap_kind {
    INFOLI_GAP_REALISTIC = 0,    /* w*dV*(0.8*exp(-dV^2/100) + 0.2) (Section 2.3.1, Alg. 1)   */
    INFOLI_GAP_SIMPLIFIED = 1    /* w*dV, a weighted accumulator (Section 2.3.2, SGJ); for
                                    UNIFORM_ALL the row sum is g*(n*Vd_i - sum_j Vd_j)      */
} infoli_gap_kind;

/* Cell state variables (structure-of-arrays order). Voltages in mV. */
enum {
    INFOLI_VD = 0,  /* dendrite voltage                       */
    INFOLI_CA = 1,  /* dendritic [Ca2+]                       */
    INFOLI_R = 2,   /* high-threshold Ca activation           */
    INFOLI_S = 3,   /* Ca-activated K activation              */
    INFOLI_Q = 4,   /* h-current activation                   */
    INFOLI_VS = 5,  /* soma voltage                           */
    INFOLI_K = 6,   /* low-threshold Ca activation            */
    INFOLI_L = 7,   /* low-threshold Ca inactivation          */
    INFOLI_H = 8,   /* soma Na inactivation                   */
    INFOLI_N = 9,   /* soma delayed-rectifier K activation    */
    INFOLI_X = 10,  /* soma K activation                      */
    INFOLI_VA = 11, /* axon voltage: the cell output          */
    INFOLI_HA = 12, /* axon Na inactivation                   */
    INFOLI_XA = 13, /* axon K activation                      */
    INFOLI_NUM_STATE = 14
};

/* The 20 per-cell conductances (mS/cm^2), area ratios and reversal
 * potentials (mV) of Table 1 ("neuron conductances: 20"), in this order:
 * g_CaH g_KCa g_h g_ld g_CaL g_Na_s g_Kdr_s g_K_s g_ls g_Na_a g_K_a g_la
 * g_int p1 p2 V_Na V_K V_Ca V_h V_L. */
enum { INFOLI_NUM_PARAMS = 20 };

/* An evoked-input pulse: amplitude (uA/cm^2, into the dendrite) added for the
 * integer steps step_begin <= n < step_end, on cells cell_begin <= i < cell_end
 * of its network (cell_end < 0 means every cell). */
typedef struct infoli_pulse {
    int64_t step_begin;
    int64_t step_end;
    float amplitude;
    int32_t cell_begin;
    int32_t cell_end;
} infoli_pulse;

enum { INFOLI_MAX_PULSES = 64 }; /* per network */

/* One network. All pointers are host pointers; NULL where marked optional. */
typedef struct infoli_network_spec {
    int32_t n_cells;            /* >= 1                                                    */
    float dt_ms;                /* > 0; the paper's step is 0.05 ms                        */
    int32_t conn;               /* infoli_conn                                             */
    float g_uniform;            /* UNIFORM_ALL weight; CSR weight when w_csr is NULL       */
    const float *w_dense;       /* DENSE: [n][n], finite                                   */
    const int64_t *row_ptr;     /* CSR: [n+1], row_ptr[0] = 0, non-decreasing, = nnz at n  */
    const int32_t *col;         /* CSR: [nnz], 0 <= col < n, strictly ascending within each
                                   row (sorted, no repeated column): else INFOLI_E_BAD_GRAPH */
    const float *w_csr;         /* CSR: [nnz] finite weights, optional                     */
    int64_t nnz;                /* CSR: number of directed edges                           */
    const float *params;        /* optional [INFOLI_NUM_PARAMS]; NULL => defaults          */
    const float *init_state;    /* optional [INFOLI_NUM_STATE][n]; NULL => rest state      */
    const float *i_bias;        /* optional [n] constant input current, uA/cm^2            */
    const infoli_pulse *pulses; /* optional [n_pulses], n_pulses <= INFOLI_MAX_PULSES      */
    int32_t n_pulses;
    const float *i_stream;      /* optional dense input [i_stream_steps][n], uA/cm^2,
                                   added at steps 0 <= n < i_stream_steps (Section 2.4.3) */
    int64_t i_stream_steps;
    int64_t step0;              /* absolute index of the first step (resume); >= 0        */
    int32_t gap_kind;           /* infoli_gap_kind; 0 (a zeroed spec) is the realistic form */
    int32_t reserved0;          /* must be 0                                               */
    const float *cell_params;   /* optional [n][INFOLI_NUM_PARAMS]: each cell's own values
                                   (Section 2.2: 20 per neuron), checked like params;
                                   NULL => params (or the defaults) for every cell. Not with
                                   PERSISTENT mode or the surrogate (INFOLI_E_UNSUPPORTED) */
} infoli_network_spec;

/* How steps are driven on the device. */
typedef enum infoli_step_mode {
    INFOLI_MODE_AUTO = 0,       /* library choice                                          */
    INFOLI_MODE_LAUNCH = 1,     /* one kernel launch per step                              */
    INFOLI_MODE_GRAPH = 2,      /* chunks of graph_chunk steps captured in a HIP graph (at
                                   init) and replayed; a remainder shorter than a chunk is
                                   launched step by step                                  */
    INFOLI_MODE_PERSISTENT = 3  /* one launch for many steps; workgroup barriers only,
                                   for networks that fit one workgroup each               */
} infoli_step_mode;

typedef struct infoli_options {
    void *hip_stream;            /* hipStream_t to queue on; NULL => context-owned stream  */
    int32_t step_mode;           /* infoli_step_mode                                       */
    int32_t graph_chunk;         /* steps per captured graph (GRAPH mode), >= 2, even      */
    int32_t max_spikes_per_cell; /* spike times kept per cell (ring); 0 => counts only     */
    int32_t tile_rows;           /* 0 => tuned; else rows per workgroup tile               */
    int32_t lanes_per_row;       /* 0 => tuned; CSR lanes per row: 4..256, power of 2     */
    int32_t check_finite;        /* 1 => a NaN/Inf state makes infoli_sync fail            */
    int32_t autotune;            /* CSR tile shapes: 0 => built-in rule; 1 => timed on the
                                    device at init, cached on disk (INFOLI_TUNE_CACHE, else
                                    ~/.cache/infoli-tune-v14.txt); 2 => timed, cache ignored */
    int32_t csr_path;            /* CSR networks: 0 => tuned choice; 1 => edge gathers;
                                    2 => coupling bitmap (one weight g, <= 16,384 cells;
                                    in the wide group when wide_threads is set);
                                    3 => Vd staged in LDS by column blocks (> 8,192 cells);
                                    4 => edge gathers from 16-byte column chunks
                                    (<= 65,536 cells); 5 => the column blocks read as one
                                    flat stream of chunks per tile (> 8,192 cells, at most
                                    8 column blocks, one weight g, network parameters, the
                                    network's first cell at a multiple of 4 in the batch's
                                    flattened cells; needs ~138 KB of LDS per workgroup,
                                    else INFOLI_E_UNSUPPORTED); other networks keep the
                                    default */
    int32_t output_ring_steps;   /* 0 => off; R > 0 => every plain step also writes the axon
                                    voltage of every cell into a device ring of R steps,
                                    read out with infoli_output_copy_async                 */
    int32_t wide_threads;        /* workgroup size of the wide launch group (all-to-all
                                    networks of >= 4,096 cells, column blocks, wide bitmap
                                    tiles): 0 => timed by the tuner (else 1024); 512 or 1024 */
    int32_t pair_path;           /* all-to-all networks with the realistic gap term:
                                    0 => library choice (each unordered pair once for a
                                    context's only network from 4,096 cells on, every
                                    ordered pair below and in batches); 1 => every
                                    ordered pair; 2 => each unordered pair once (the pair
                                    term of Section 2.3.1, Algorithm 1, is odd in dV,
                                    so the pair (j, i) gives minus the term of (i, j)).
                                    Once costs
                                    64 x (B/2 + waves + 1) x B floats of partial sums per
                                    network of B = ceil(n/64) blocks (8.4 MB at 16,384
                                    cells). With the simplified term (the closed form of
                                    Section 2.3.2 needs the sum of all voltages): 0 =>
                                    that sum once per step by a separate kernel for a
                                    context's only network from 12,288 cells on, else by
                                    every tile; 1 => by every tile; 2 => once per step
                                    (8 bytes per 4,096 cells)                              */
} infoli_options;

typedef struct infoli_ctx infoli_ctx;

/* Fill *opt with the defaults (AUTO mode, 64 spike times, autotuned tiles,
 * checks on). */
infoli_status infoli_default_options(infoli_options *opt);

/* Copy the default cell parameters (see INFOLI_NUM_PARAMS) into out[20]. */
infoli_status infoli_default_params(float *out);

/* Rest state of one cell: every voltage at v0_mv, every gate at its steady
 * state there, [Ca2+] at its steady state. params NULL => defaults.
 * out[INFOLI_NUM_STATE]. */
infoli_status infoli_rest_state(const float *params, float v0_mv, float *out);

/* Create a context for one network: validates the spec, copies every array
 * to the device and prepares the step kernels. On failure *out = NULL. */
infoli_status infoli_init(const infoli_network_spec *spec, const infoli_options *opt,
                          infoli_ctx **out);

/* Create a context for n_instances independent networks of any sizes and
 * connectivities, stepped together by the same launches. Instance k's cells
 * are numbered 0..n_cells-1 within the instance. All specs share step0. */
infoli_status infoli_batch_init(const infoli_network_spec *specs, int32_t n_instances,
                                const infoli_options *opt, infoli_ctx **out);

/* Queue n_steps synchronous steps (n_steps >= 0). Returns without waiting. */
infoli_status infoli_step(infoli_ctx *ctx, int64_t n_steps);

/* Wait for queued work. Returns INFOLI_E_NUMERIC if check_finite is on and a
 * state value became non-finite. */
infoli_status infoli_sync(infoli_ctx *ctx);

/* Blocking copy of instance `instance`'s state to host_soa
 * ([INFOLI_NUM_STATE][n], capacity cap_floats) and of the absolute step
 * index reached to *step_out (optional). */
infoli_status infoli_read_state(infoli_ctx *ctx, int32_t instance, float *host_soa,
                                int64_t cap_floats, int64_t *step_out);

/* Like infoli_read_state, into device memory dev_soa (>= 14*n floats) on
 * the context's stream, without waiting. */
infoli_status infoli_read_state_device(infoli_ctx *ctx, int32_t instance, float *dev_soa);

/* Replace instance `instance`'s state and set the absolute step index of all
 * instances to `step` (resume: a run split at step k and continued from the
 * state read there matches the straight run bitwise). */
infoli_status infoli_write_state(infoli_ctx *ctx, int32_t instance, const float *host_soa,
                                 int64_t step);

/* Gap currents I_gap,i (uA/cm^2) of every cell of the instance, computed from
 * the current Vd by the same kernel code the step uses. Blocking. host[n]. */
infoli_status infoli_read_gap_current(infoli_ctx *ctx, int32_t instance, float *host,
                                      int64_t cap);

/* Spikes of the instance: counts[n] (upward 0 mV crossings of Va) and, when
 * times_ms is not NULL, the last max_spikes_per_cell spike times of each cell,
 * times_ms[i * max_spikes_per_cell + (k mod max_spikes_per_cell)] for its k-th
 * spike (linear interpolation between steps, ms from step 0). Blocking. */
infoli_status infoli_read_spikes(infoli_ctx *ctx, int32_t instance, int32_t *counts,
                                 int64_t counts_cap, float *times_ms, int64_t times_cap);

/* Reset spike counts and times to zero. */
infoli_status infoli_clear_spikes(infoli_ctx *ctx);

/* Description of what the context runs. */
/* Output streaming (Section 2.4.3: the host receives each step's output, the
 * axon voltages, while later steps compute, over a second stream). Requires
 * options.output_ring_steps = R > 0. The output of step s is Va of every cell
 * after step s (the state of step s + 1), held in ring slot s mod R until
 * step s + R overwrites it.
 *
 * infoli_output_copy_async queues, on the context's copy stream, the copy of
 * the outputs of steps [step_begin, step_begin + n_steps) into
 * host[n_steps][total_cells] (cells in batch order: instance 0's cells, then
 * instance 1's, ...), ordered after the steps that produce them; it returns
 * before the copy is done. Steps queued later that would overwrite slots of
 * a pending copy wait for it on the device. host must hold
 * cap_floats >= n_steps * total_cells floats and stay valid until
 * infoli_output_wait returns; pinned memory (hipHostMalloc) lets the copy
 * overlap the compute, pageable memory works but is staged. Errors
 * (INFOLI_E_INVALID_ARG): no ring, n_steps < 1 or > R, steps not yet queued
 * (step_begin + n_steps > the context's step count), steps already
 * overwritten (step_begin < step count - R) or before the context's first
 * step, host NULL or too small. The surrogate's macro steps do not write the
 * ring (infoli_step_surrogate refuses a context that has one). */
infoli_status infoli_output_copy_async(infoli_ctx *ctx, int64_t step_begin, int64_t n_steps, float *host,
                                       int64_t cap_floats);

/* Block the calling thread until every queued output copy has completed. */
infoli_status infoli_output_wait(infoli_ctx *ctx);

typedef struct infoli_info {
    int32_t n_instances;
    int64_t total_cells;
    int64_t pairs_per_step;     /* directed gap pair-interactions evaluated per step    */
    int64_t step;               /* absolute step index reached (after queued work)     */
    int32_t step_mode;          /* mode in use                                          */
    int32_t n_tiles;            /* workgroups per step launch                           */
    int32_t tile_rows;          /* rows per tile of the largest instance               */
    int32_t lanes_per_row;
    int64_t device_bytes;       /* device memory held                                   */
    int32_t tuned;              /* networks whose tile shapes were timed at init        */
    int32_t tune_cached;        /* networks whose tile shapes came from the cache       */
    int32_t n_tiles_wide;       /* of n_tiles, those in 1024-thread workgroups (a second
                                   launch per step, concurrent with the first)          */
    int32_t n_bitmap;           /* CSR networks on the coupling-bitmap path             */
    int32_t n_blocked;          /* CSR networks on the column-blocked path              */
    int32_t wide_threads;       /* workgroup size of the wide launch group (512 or 1024) */
    int32_t n_stream;           /* CSR networks on the chunk stream (CSR_STREAM path)    */
    int32_t tune_mode;          /* whole-step launch arrangement the tuner chose, -1 when
                                   the shapes were not tuned (bits: 1 every class in its
                                   256-thread shape, 2 launch groups one after the other,
                                   4 no chunked 256-thread gathers, 8 every class in its
                                   1024-thread shape, 16 wide group of 512 threads, 32
                                   every class with a bitmap shape on it)                 */
    int32_t stream_round;       /* chunks per round of the chunk stream networks (the
                                   largest; 8,192 or 4,096 as the tuner timed), 0 none    */
    int32_t n_sym;              /* all-to-all networks taking each unordered pair once,
                                   or (simplified term) their voltage sum once per step  */
} infoli_info;
infoli_status infoli_get_info(const infoli_ctx *ctx, infoli_info *info);

/* The gap-junction path one network runs, as chosen at init (by the tuner or
 * the built-in rule), which fixes the form in which its coupling is read each
 * step (the coupling of Section 2.3, Algorithm 1; for the CSR paths, the
 * same sum over each row's neighbours, reordered only within a row):
 *   NONE        no gap junctions;
 *   UNIFORM     all-to-all with one weight: only the Vd vector is read;
 *   DENSE       the n x n fp32 weight matrix;
 *   CSR_GATHER  row pointers and columns (uint16 when every CSR network of the
 *               context has <= 65,536 cells, else int32), fp32 weights if given;
 *   CSR_CHUNKED the same columns as uint16 in 16-byte chunks of eight;
 *   CSR_BITMAP  one bit per (row, column) pair; every pair is evaluated and
 *               masked by its bit (one weight g, <= 16,384 cells);
 *   CSR_STREAM  the CSR_CHUNKED columns of each column block (relative to
 *               the block) as one contiguous run per tile, plus one byte per
 *               chunk naming its row (Vd staged block by block).
 *   UNIFORM_SYM all-to-all, each unordered pair once: a separate kernel
 *               writes per-block partial sums, the step adds them per cell
 *               in a fixed order (option pair_path).
 *   UNIFORM_SUM all-to-all with the simplified term: a separate kernel
 *               writes fp64 sums of the voltages of each 4,096 cells, and
 *               every tile adds those instead of all n voltages (option
 *               pair_path).
 * (The persistent step mode walks CSR rows from the gather format.)
 * *path receives the code; *vd_blocked (either pointer may be NULL) receives
 * 1 when the network's Vd is staged in LDS one column block at a time (CSR
 * networks too large for one LDS copy), else 0.
 * Errors: INVALID_ARG when ctx is NULL or instance is out of range. */
typedef enum infoli_gap_path {
    INFOLI_PATH_NONE = 0,
    INFOLI_PATH_UNIFORM = 1,
    INFOLI_PATH_DENSE = 2,
    INFOLI_PATH_CSR_GATHER = 3,
    INFOLI_PATH_CSR_CHUNKED = 4,
    INFOLI_PATH_CSR_BITMAP = 5,
    INFOLI_PATH_CSR_STREAM = 6,
    INFOLI_PATH_UNIFORM_SYM = 7,
    INFOLI_PATH_UNIFORM_SUM = 8
} infoli_gap_path;
infoli_status infoli_get_gap_path(const infoli_ctx *ctx, int32_t instance, int32_t *path, int32_t *vd_blocked);

/* Duration (ms, HIP events on the context stream) of the last infoli_step
 * call's device work; valid after infoli_sync. */
infoli_status infoli_last_step_ms(infoli_ctx *ctx, float *ms);

/* ------------------------------------------------------------------ surrogate
 * A learned surrogate of the cell update: an MLP 16 -> 128 -> 128 -> 16 with
 * SiLU, BF16 weights on the matrix cores and FP32 accumulation, mapping a
 * cell's normalised [14 state variables, I_gap, I_app] to its normalised state
 * increment over a macro step of 4 time steps, during which the gap current
 * (computed exactly in fp32 at the macro step's start) and the input are held.
 * The plain method stays the fallback and the reference (drift check). This part
 * is not in the paper; it serves callers that trade a bounded error for speed.
 *
 * Parameters: INFOLI_MLP_PARAMS fp32 values in the order W1[128][16] b1[128]
 * W2[128][128] b2[128] W3[16][128] b3[16] (W[out][in]). Normalisation: 64
 * floats in_mean[16] in_rstd[16] out_mean[16] out_std[16] (features: the 14
 * state variables, I_gap, I_app; outputs: the 14 increments, 2 pads). */
enum { INFOLI_MLP_PARAMS = 20752 };

typedef struct infoli_train_cfg {
    int64_t n_transitions;      /* training-set size (rounded up to whole trajectories)   */
    int32_t n_trajectories;     /* independent cells generating it                        */
    int32_t burn_in;            /* unrecorded macro steps per trajectory: uniform in
                                   [0, burn_in] (covers the slow variables' excursion)     */
    int32_t batch;              /* samples per optimiser step, multiple of 64             */
    int32_t steps;              /* optimiser steps                                        */
    float lr, beta1, beta2, eps;/* Adam; the rate decays from lr to lr_min (cosine)        */
    float lr_min;
    float v_max;                /* the surrogate's regime: transitions are recorded only
                                   when they start with Vd, Vs, Va <= v_max (mV, >= -50)   */
    float bias_sd;              /* per-trajectory constant input ~ N(0, bias_sd^2)        */
    float gap_sd, gap_rho;      /* AR(1) gap current: stationary sd, lag-1 correlation    */
    float pulse_p;              /* pulse start probability per macro step                 */
    float pulse_lo, pulse_hi;   /* pulse amplitude ~ U[lo, hi] uA/cm^2                    */
    int32_t pulse_len;          /* pulse length in macro steps                            */
    float ca_max;               /*   and [Ca] <= ca_max (above the rest value); the same
                                   bounds as infoli_drift_cfg's                            */
    uint64_t seed;              /* counter-based draws of the data and the batches        */
    const float *init_params;   /* [INFOLI_MLP_PARAMS] initial weights (host), required   */
} infoli_train_cfg;

typedef struct infoli_train_report {
    int64_t n_transitions;
    int32_t steps;
    float loss_first, loss_last;  /* mean squared error of the normalised increments     */
    float data_ms, train_ms;      /* device time: data generation, optimisation          */
} infoli_train_report;

enum { INFOLI_SURROGATE_MLP = 0,        /* MLP with drift check and plain fallback        */
       INFOLI_SURROGATE_PLAIN_HOLD = 1  /* every cell by the plain method, gap held 4 dt  */ };

typedef struct infoli_drift_cfg {
    float theta_mv;             /* a checked cell whose MLP voltages differ from the plain
                                   ones by more than this (mV) is flagged                 */
    float v_max;                /* regime served by the MLP: Vd, Vs, Va <= v_max (mV)     */
    int32_t sample_every;       /* checked cells per macro step: 1 in sample_every; 0 = none */
    int32_t hold_steps;         /* macro steps a flagged cell stays on the plain method   */
    int32_t mode;               /* INFOLI_SURROGATE_*                                     */
    float z_max;                /* a cell with a normalised MLP input beyond +-z_max is
                                   guarded (0: no bound)                                  */
    float ca_max;               /*   and [Ca] <= ca_max                                   */
} infoli_drift_cfg;

typedef struct infoli_drift_report {
    int64_t plain_cell_macro_steps;  /* cell macro steps advanced by the plain method     */
    int64_t checked;                 /* drift checks made                                 */
    int64_t flagged;                 /* checks past theta                                 */
    int64_t guarded;                 /* cell macro steps sent to the plain method by the
                                        guards: a cell outside the regime (v_max, ca_max),
                                        an input beyond z_max, or an MLP candidate with a
                                        voltage above v_max or beyond +-150 mV (or not
                                        finite)                                          */
    float ms;                        /* device time of the call                           */
} infoli_drift_report;

infoli_status infoli_default_train_cfg(infoli_train_cfg *cfg);
infoli_status infoli_default_drift_cfg(infoli_drift_cfg *cfg);

/* Generate the training set on the device (the context's single network's
 * cell parameters; independent cells under random currents advanced by the
 * plain method), normalise it, and train the MLP with Adam. loss_hist
 * (optional, [cfg->steps]) receives the loss of every step. Blocking. */
infoli_status infoli_surrogate_train(infoli_ctx *ctx, const infoli_train_cfg *cfg,
                                     infoli_train_report *report, float *loss_hist);

/* Copy out (either pointer may be NULL) or install trained weights and
 * normalisation (params [INFOLI_MLP_PARAMS], norm [64]; scales > 0). */
infoli_status infoli_surrogate_get(infoli_ctx *ctx, float *params, float *norm);
infoli_status infoli_surrogate_set(infoli_ctx *ctx, const float *params, const float *norm);

/* Advance n_macro macro steps of 4 time steps each (single-network contexts).
 * A cell takes the MLP unless it is held, checked or guarded (see the report's
 * fields); a checked cell runs the plain method and is flagged when the MLP's
 * voltages differ from it by more than theta; a flagged cell is held on the
 * plain method for hold_steps macro steps.
 * cfg NULL => defaults (theta 0.5 mV, v_max -40 mV, ca_max 20, 1/64 checked per
 * macro step, 50 macro steps of hold, z_max 8). report optional (blocking when
 * given). */
infoli_status infoli_step_surrogate(infoli_ctx *ctx, int64_t n_macro, const infoli_drift_cfg *cfg,
                                    infoli_drift_report *report);

/* The MLP kernels on host data, blocking: forward y[batch][16] of x[batch][16];
 * loss (mean over the batch and the first 14 outputs of the squared error) and
 * its gradient grad[INFOLI_MLP_PARAMS]; one Adam step on params/m/v in place
 * (bias correction with step t >= 1). batch: multiple of 16. */
infoli_status infoli_mlp_forward(const float *params, const float *x, int32_t batch, float *y);
infoli_status infoli_mlp_loss_grad(const float *params, const float *x, const float *t, int32_t batch,
                                   float *loss, float *grad);
infoli_status infoli_mlp_adam_step(float *params, float *m, float *v, const float *grad, int64_t t,
                                   float lr, float beta1, float beta2, float eps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the loss and
 * gradient of infoli_mlp_loss_grad on device data, queued on `stream`
 * (a hipStream_t; NULL = the null stream) and not waited for. Same kernels
 * and summation order, so the results equal infoli_mlp_loss_grad's bit for
 * bit.
 *   d_params [INFOLI_MLP_PARAMS], d_x and d_t [batch][16] row-major fp32,
 *   d_grad [INFOLI_MLP_PARAMS] (written), d_loss [1] (written; may be NULL):
 *   device memory of the current device, owned by the caller, left in place
 *   until the queued work has run.
 *   batch: a multiple of 16, at most 8192 (else INFOLI_E_INVALID_ARG, with
 *   the limit in the message). Host or other-device pointers:
 *   INFOLI_E_INVALID_ARG; nothing is queued on any error.
 * The call allocates nothing: its staging (bf16 weights, split-K partial
 * gradients, transposed activations; 10,284,800 bytes) is a static device
 * array that each GPU holds from the first call on it until the process
 * ends. Every call on one GPU uses that one array: calls whose queued work
 * overlaps on a GPU (two streams, two threads) race and give wrong results;
 * serialise them. Each call writes all the staging it reads, so nothing
 * from an earlier call carries over. The parameters are not checked for
 * NaN or infinity (they stay on the device). */
infoli_status infoli_mlp_loss_grad_noalloc(const float *d_params, const float *d_x, const float *d_t,
                                           int32_t batch, float *d_loss, float *d_grad, void *stream);

/* Names of state variables ("Vd", "Ca", ...); NULL when out of range. */
const char *infoli_state_var_name(int32_t v);

/* Last error message of ctx, or of the calling thread's last failed call
 * when ctx is NULL. Never NULL. */
const char *infoli_last_error(const infoli_ctx *ctx);

/* Free the context and all its device memory. NULL is allowed. */
void infoli_destroy(infoli_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* INFOLI_API_H_ */
