// One synchronous simulation step for a list of tiles (Section 2.2): every
// workgroup takes one tile = a block of consecutive cells of one network,
// computes their gap-junction currents from the step-n dendritic voltages
// (Section 2.3, Algorithm 1) and then their compartment update into the
// step-n+1 buffer. Reads only the step-n buffer and writes only the step-n+1
// buffer, so the kernel boundary is the step barrier.
//
// Gap-current layouts (per network):
//   UNIFORM_ALL  lanes = receiving cells (64 per tile); the waves of the
//                workgroup split the sending cells j, whose prescaled Vd is
//                staged in LDS in chunks and read as wave-wide broadcasts.
//                w = g is factored out and the linear part 0.2*sum_j dV is
//                taken in closed form, 0.2*(n*Vd_i - sum_j Vd_j), in fp64.
//   DENSE        lanes = sending cells j of one row (coalesced weight rows),
//                one row per wave at a time, butterfly reduction.
//   BITMAP       (CSR networks with one weight g, when faster) the coupling
//                pattern as one bit per pair: 16 receiving cells per wave,
//                four lane groups per cell take interleaved 32-sender blocks
//                of a 128-sender group (conflict-free LDS rows), waves split
//                the groups; every pair is evaluated and masked.
//   BLOCKED CSR  (networks too large for one LDS copy of Vd) Vd is staged in
//                LDS one column block at a time; each row's edges of that
//                block (precomputed offsets, columns sorted) gather from LDS;
//                partial sums stay in registers across blocks.
//   CSR          groups of L lanes per row stride over the row's edges and
//                gather Vd of the neighbours, from a copy of the network's
//                Vd staged in LDS when the tile's edges outnumber the cells,
//                else from global memory; columns are 16-bit when every
//                network has at most 65,536 cells. Butterfly reduction per
//                group.
// Every reduction has a fixed order: results are bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

#include "cell_model.hpp"

namespace infoli {

enum : int { CONN_NONE = 0, CONN_UNIFORM = 1, CONN_DENSE = 2, CONN_CSR = 3 };

constexpr int kMaxTileRows = 256;   // rows (cells) per tile, any layout (<= BLOCK)
constexpr int kUniformRows = 64;    // rows per UNIFORM_ALL tile (one per lane)
constexpr int kChunk = 8192;        // Vd values staged in LDS per pass
constexpr int kBatch = 16;          // CSR edges per lane per batch of loads

// log2(e)/100: exp(-dV^2/100) = 2^(-(dV*a)^2) with a = sqrt(log2(e)/100).
constexpr float kL2eOver100 = 0.014426950408889634f;
constexpr float kPreScale = 0.12011224087864498f;      // sqrt(log2(e)/100)
constexpr float kInvPreScale = 8.325546111576977f;     // 1/kPreScale
constexpr float kSentinel = 1.0e19f;                   // prescaled pad: term == -0

struct InstDesc {
    int64_t cell_off;      // flattened index of the network's cell 0
    int64_t rp_off;        // CSR: offset of the network's row_ptr[0]
    int64_t w_off;         // DENSE: offset of w[0][0]; CSR: offset of edge 0
    int64_t stream_off;    // offset of the network's dense input stream, -1 none
    int64_t stream_steps;
    int32_t n;
    int32_t conn;
    float g;
    int32_t has_w;         // CSR: per-edge weights present
    int32_t pulse_off;
    int32_t n_pulses;
    int32_t lanes_per_row; // CSR: lanes per row (4..64)
    int32_t vd_lds;        // CSR: stage the network's Vd in LDS (n <= kChunk)
    int32_t col16;         // CSR: columns stored as uint16
    int32_t bitmap;        // CSR with uniform g: gap from the coupling bitmap
    int32_t blocked;       // CSR: Vd staged in LDS one column block at a time
    int32_t nblk;          // blocked: number of column blocks
    int32_t wide;          // bitmap: run in the 1024-thread launch group
    int32_t chunked;       // CSR gathers from the chunked rows layout
    int32_t sgj;           // simplified (linear) gap junctions: term w * dV
    int32_t pcell;         // per-cell parameters in StepArgs::cparams
    int32_t stream;        // blocked: the flat chunk stream (row tags) instead of row groups
    int32_t sym;           // UNIFORM: sums a kernel ahead of the step wrote into psym: each
                           // unordered pair once (k_pairs_sym), or for the simplified term the
                           // voltage sum (k_vsum)
    int64_t bits_off;      // bitmap: offset of the network's first word
    int64_t blk_off;       // blocked: offset of the network's [n][nblk] block starts
    int64_t ca_off;        // chunked rows: offset of the [n + 1] row chunk starts, -1 none
    int64_t chk_off;       // chunked rows: first chunk of the network
    int64_t cb_off;        // chunked blocks: offset of the [n][nblk + 1] chunk starts, -1 none
    int64_t chkb_off;      // chunked blocks: first chunk of the network
    int64_t psym_off;      // sym: offset of the network's partial sums in StepArgs::psym
    int32_t sym_ki;        // sym: row blocks per workgroup of k_pairs_sym
    int32_t stream_round;  // stream: chunks per round (0: kStreamRound)
    CellParams p;
};

struct Tile {
    int32_t inst;
    int32_t row0;
    int32_t row1;
    int32_t pad0;
};

struct DevPulse {
    int64_t n0, n1;        // active for steps n0 <= step < n1
    float amp;
    int32_t c0, c1;        // on local cells c0 <= i < c1
    int32_t pad0;
};

struct StepArgs {
    const InstDesc* inst;
    const Tile* tiles;
    const DevPulse* pulses;
    const float* bias;         // [cells]
    const int64_t* row_ptr;    // CSR row pointers of all networks
    const int32_t* col;        // CSR columns (local cell index)
    const uint16_t* col16;     // CSR columns, 16-bit form
    const uint32_t* bits;      // coupling bitmaps
    const int32_t* blk;        // blocked CSR: per row, first edge of each column block
    int32_t blk_cols;          // blocked CSR: cells per column block
    const int32_t* ca;         // chunked rows: per row, first chunk (relative to the network's)
    const int32_t* cb;         // chunked blocks: per row and block, first chunk
    const uint4* chk;          // chunks of eight 16-bit columns
    const float* chkw;         // per-edge weights in the chunk layout (8 per chunk)
    const uint8_t* rtag;       // chunked blocks: per chunk, its row mod 256
    const float* w;            // DENSE matrices and CSR weights
    const float* i_stream;     // dense input streams
    int32_t* spike_count;      // [cells]
    float* spike_times;        // [cells][spike_cap]
    int32_t* flags;            // [0]: non-finite state seen
    float* igap_out;           // gap-only mode: [cells]
    unsigned int* list_reset;  // when set, workgroup 0 zeroes it (the surrogate's plain-cell list)
    const int64_t* d_step;     // when set, step = *d_step + step offset
    int64_t stride;            // state row stride (floats)
    float dt;
    int32_t spike_cap;
    int32_t gap_only;
    int32_t dry;               // timing runs: write the next state only
    int32_t out_slots;         // output ring: slots (steps), 0 => none
    float* out_ring;           // [out_slots][stride]: Va after step s in slot s mod out_slots
    const float* cparams;      // [20][stride]: per-cell parameters (networks with pcell)
    const float* psym;         // partial row sums of the sym networks (k_pairs_sym)
};

// The parameters of one cell: the network's, or the cell's own (SoA rows).
__device__ __forceinline__ CellParams cell_params_of(const StepArgs& a, const InstDesc& d, int64_t cell) {
    CellParams p = d.p;
    if (d.pcell) {
        float* f = reinterpret_cast<float*>(&p);
#pragma unroll
        for (int v = 0; v < 20; ++v) f[v] = a.cparams[v * a.stride + cell];
    }
    return p;
}

// Output ring slot of step s (s >= 0).
__device__ __forceinline__ int64_t out_slot(const StepArgs& a, int64_t s) {
    return (s % a.out_slots) * a.stride;
}

__device__ __forceinline__ float wave_sum_xor(float v, int width) {
    // butterfly over `width` consecutive lanes (power of two <= 64)
    for (int m = width >> 1; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ float gap_factor(float dv) {
    // 0.8*exp(-dv^2/100) + 0.2 via the hardware 2^x
    return fmaf(0.8f, __builtin_amdgcn_exp2f(-(dv * dv) * kL2eOver100), 0.2f);
}

// The same factor of a voltage difference prescaled by kPreScale (Vd staged
// in LDS times sqrt(log2(e)/100)): 0.8 * 2^(-dv'^2) + 0.2; the sum over a row
// is scaled back by kInvPreScale once.
__device__ __forceinline__ float gap_factor_ps(float dvs) {
    return fmaf(0.8f, __builtin_amdgcn_exp2f(-(dvs * dvs)), 0.2f);
}

// The factor multiplying w * dV: the realistic one (of a prescaled
// difference when PS), or 1 for simplified gap junctions (Section 2.3.2),
// which is linear, so a prescaled row sum scales back the same way.
template <bool SGJ, bool PS>
__device__ __forceinline__ float pair_factor(float dv) {
    if constexpr (SGJ) return 1.0f;
    else return PS ? gap_factor_ps(dv) : gap_factor(dv);
}

// Blocks of the all-to-all path that takes each unordered pair once
// (k_pairs_sym below).
constexpr int kSymCells = 4096;     // all-to-all networks from this size on (library choice)
constexpr int kSymMaxKi = 16;       // row blocks per workgroup, at most

__host__ __device__ constexpr int sym_blocks(int n) { return (n + 63) / 64; }
__host__ __device__ constexpr int sym_kmax(int n) { return sym_blocks(n) / 2; }
__host__ __device__ constexpr int sym_shares(int n, int ki) {       // workgroups per column block
    return sym_kmax(n) > ki ? (sym_kmax(n) + ki - 1) / ki : 1;
}
// floats of a network's partial sums: [B][K][64] row sums of block pairs,
// [B][S][64] column sums, [B][64] own-block row sums, then B fp64 sums of
// each block's voltages (a multiple of 64 floats in all)
__host__ __device__ constexpr int64_t sym_vsum_off(int n, int ki) {
    return (int64_t)sym_blocks(n) * 64 * (sym_kmax(n) + sym_shares(n, ki) + 1);
}
__host__ __device__ constexpr int64_t sym_floats(int n, int ki) {
    return (sym_vsum_off(n, ki) + 2 * (int64_t)sym_blocks(n) + 63) / 64 * 64;
}

// The simplified term's closed form g (n Vd_i - sum_j Vd_j) needs one sum of
// all voltages. Each tile adding all n of them is O(n^2 / 64) loads per
// step; from kSgjSumCells cells on, a context's only such network has k_vsum
// write one fp64 sum per kVsumCells cells ahead of the step instead (one
// more launch; measured 0.1 us slower per step at 8,192 cells, 1.0 us faster
// at 12,288).
constexpr int kVsumCells = 4096;
constexpr int kSgjSumCells = 12288;
__host__ __device__ constexpr int vsum_groups(int n) { return (n + kVsumCells - 1) / kVsumCells; }
__host__ __device__ constexpr int64_t vsum_floats(int n) { return (2 * (int64_t)vsum_groups(n) + 63) / 64 * 64; }

template <int BLOCK>
__device__ __forceinline__ void gap_uniform(const StepArgs& a, const InstDesc& d, const Tile& t,
                                            const float* __restrict__ vd, float* s_ig,
                                            float4* s_v4, float* s_part, double* s_red) {
    constexpr int W = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nrows = t.row1 - t.row0;
    const int n = d.n;
    const bool valid = lane < nrows;
    const float vi = valid ? vd[t.row0 + lane] : 0.0f;
    const float vis = vi * kPreScale;
    float* s_v = reinterpret_cast<float*>(s_v4);
    float acc0 = 0.0f, acc1 = 0.0f;
    double vsum = 0.0;
    if (d.sgj) {
        // simplified: g (n Vd_i - sum_j Vd_j), the sum in fp64
        for (int k = threadIdx.x; k < n; k += BLOCK) vsum += (double)vd[k];
    } else if (d.sym) {
        // the realistic form's linear part from the blocks' sums k_pairs_sym wrote
        const double* bs = reinterpret_cast<const double*>(a.psym + d.psym_off + sym_vsum_off(n, d.sym_ki));
        for (int k = threadIdx.x; k < sym_blocks(n); k += BLOCK) vsum += bs[k];
    }
    if (d.sym && !d.sgj && valid) {
        // the row's partial sums from k_pairs_sym, in a fixed order: its
        // block's own pairs, its row sums of block pairs (k = 1 .. KR), the
        // column sums of its block; each wave adds a consecutive run,
        // loading a batch at a time so that the loads overlap
        const int r = t.row0 + lane, R = r >> 6, l = r & 63;
        const int B = sym_blocks(n), K = sym_kmax(n), S = sym_shares(n, d.sym_ki);
        const int KR = (B & 1) ? (B - 1) / 2 : B / 2 - 1 + (R >= B / 2 ? 1 : 0);
        const float* P = a.psym + d.psym_off;
        const float* prow = P + (int64_t)R * K * 64 + l;
        const float* pcol = P + (int64_t)B * K * 64 + (int64_t)R * S * 64 + l;
        const float* pdiag = P + (int64_t)B * K * 64 + (int64_t)B * S * 64 + (int64_t)R * 64 + l;
        const int E = 1 + KR + S, per = (E + W - 1) / W;
        const int q0 = wave * per, q1 = min(E, q0 + per);
        constexpr int kQ = 16;
        for (int qb = q0; qb < q1; qb += kQ) {
            float v[kQ];
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                const int q = qb + u;
                v[u] = q >= q1 ? 0.0f : q == 0 ? *pdiag : q <= KR ? prow[(int64_t)(q - 1) * 64]
                                                                   : pcol[(int64_t)(q - 1 - KR) * 64];
            }
#pragma unroll
            for (int u = 0; u < kQ; ++u) acc0 += v[u];
        }
    }
    for (int c0 = 0; c0 < (d.sgj || d.sym ? 0 : n); c0 += kChunk) {
        const int cn = min(kChunk, n - c0);
        // per-wave share, a multiple of 8 values; the tail is padded with a
        // sentinel whose term is exactly -0
        const int per = (((cn + W - 1) / W) + 7) & ~7;
        __syncthreads();
        for (int k = threadIdx.x; k < W * per; k += BLOCK) {
            if (k < cn) {
                const float v = vd[c0 + k];
                s_v[k] = v * kPreScale;
                vsum += (double)v;
            } else {
                s_v[k] = kSentinel;
            }
        }
        __syncthreads();
        const float4* p = s_v4 + (wave * per) / 4;
        for (int q = 0; q < per / 4; q += 2) {
            const float4 u = p[q];
            const float4 v = p[q + 1];
            float d0 = vis - u.x, d1 = vis - u.y, d2 = vis - u.z, d3 = vis - u.w;
            acc0 = fmaf(d0, __builtin_amdgcn_exp2f(-(d0 * d0)), acc0);
            acc1 = fmaf(d1, __builtin_amdgcn_exp2f(-(d1 * d1)), acc1);
            acc0 = fmaf(d2, __builtin_amdgcn_exp2f(-(d2 * d2)), acc0);
            acc1 = fmaf(d3, __builtin_amdgcn_exp2f(-(d3 * d3)), acc1);
            d0 = vis - v.x; d1 = vis - v.y; d2 = vis - v.z; d3 = vis - v.w;
            acc0 = fmaf(d0, __builtin_amdgcn_exp2f(-(d0 * d0)), acc0);
            acc1 = fmaf(d1, __builtin_amdgcn_exp2f(-(d1 * d1)), acc1);
            acc0 = fmaf(d2, __builtin_amdgcn_exp2f(-(d2 * d2)), acc0);
            acc1 = fmaf(d3, __builtin_amdgcn_exp2f(-(d3 * d3)), acc1);
        }
    }
    s_part[wave * 64 + lane] = acc0 + acc1;
    // fixed-order reduction of sum_j Vd_j (fp64)
    for (int m = 32; m > 0; m >>= 1) vsum += __shfl_xor(vsum, m, 64);
    if (lane == 0) s_red[wave] = vsum;
    __syncthreads();
    if (threadIdx.x < 64 && valid) {
        float e = 0.0f;
        for (int w = 0; w < W; ++w) e += s_part[w * 64 + lane];
        double tot = 0.0;
        for (int w = 0; w < W; ++w) tot += s_red[w];
        const float lin = (float)((double)n * (double)vi - tot);
        s_ig[lane] = d.sgj ? d.g * lin : d.g * (0.8f * (e * kInvPreScale) + 0.2f * lin);
    }
}

// The simplified all-to-all form with the voltage sum taken once per step:
// the workgroup adds the fp64 group sums k_vsum wrote in a fixed order, then
// each of the tile's rows (up to kMaxTileRows) takes g (n Vd_i - sum).
template <int BLOCK>
__device__ __forceinline__ void gap_uniform_sum(const StepArgs& a, const InstDesc& d, const Tile& t,
                                                const float* __restrict__ vd, float* s_ig, double* s_red) {
    constexpr int W = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const double* gs = reinterpret_cast<const double*>(a.psym + d.psym_off);
    double vsum = 0.0;
    for (int k = threadIdx.x; k < vsum_groups(d.n); k += BLOCK) vsum += gs[k];
    for (int m = 32; m > 0; m >>= 1) vsum += __shfl_xor(vsum, m, 64);
    if (lane == 0) s_red[wave] = vsum;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < W; ++w) tot += s_red[w];
    for (int k = threadIdx.x; k < t.row1 - t.row0; k += BLOCK)
        s_ig[k] = d.g * (float)((double)d.n * (double)vd[t.row0 + k] - tot);
}

// ---------------------------------------------------------------- all-to-all, each unordered pair once
// The pair term dV * f(dV) (Section 2.3.1, Algorithm 1) is odd in dV, and
// exactly so in floating point:
// the difference of (j, i) is minus that of (i, j), its square and the
// factor are the same, so its term is minus the other. An all-to-all
// network with one weight g therefore needs each unordered pair once.
// Cells form blocks of 64 (B blocks; the last one padded with kSentinel,
// whose terms against any cell are zero). The pairs of distinct blocks
// {J, J + k mod B}, 1 <= k <= B / 2 (k = B / 2 only for J < B / 2 when B is
// even, so that each block pair is taken once), belong to column block J.
// A workgroup of four waves takes sym_ki row blocks I = J + k in turn,
// lanes being I's cells, each wave with 16 of J's voltages in scalar
// registers: per pair one difference, square, exponential and two fused
// multiply-adds, one into the row's sum (the four waves' parts added in LDS,
// written for (I, k)) and one into the column's (added over the row blocks,
// then over the lanes). Each block's own 64 x 64 ordered pairs give its row
// sums directly. The step adds a cell's partial sums in a fixed order, so
// results do not depend on scheduling.

// Halving step of a lane-transposed sum: v[0 .. 2H) are sums of 2H
// consecutive columns over this lane; afterwards v[0 .. H) hold the sums over
// this lane and lane ^ H of the half of them selected by bit H of the lane.
// After H = 8, 4, 2, 1 a lane holds column (lane & 15)'s sum over the 16
// lanes that share its bits 4 and 5.
template <int H>
__device__ __forceinline__ void sym_halve(float* v, int lane) {
    const bool hi = (lane & H) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const float send = hi ? v[i] : v[i + H];
        const float keep = hi ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, H, 64);
    }
}

// One workgroup of four waves per (column block J, share s of its row
// blocks); wave w takes J's columns 16w .. 16w + 15 in scalar registers.
// Per row block the four waves' row sums meet in LDS and are added in wave
// order. vd: the network's Vd row; P: its partial sums.
static __global__ __launch_bounds__(256) void k_pairs_sym(const float* __restrict__ vd, int n, int ki,
                                                          float* __restrict__ P) {
    __shared__ float s_row[4][kSymMaxKi + 1][64];
    const int B = sym_blocks(n), K = sym_kmax(n), S = sym_shares(n, ki);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int g = blockIdx.x;
    if (g >= B * S) return;
    const int J = g / S, s = g - J * S;
    float* prow = P;                                   // [B][K][64]
    float* pcol = P + (int64_t)B * K * 64;             // [B][S][64]
    float* pdiag = pcol + (int64_t)B * S * 64;         // [B][64]
    double* bsum = reinterpret_cast<double*>(P + sym_vsum_off(n, ki));   // [B]
    const int cj = J * 64 + lane;
    const float vraw = cj < n ? vd[cj] : 0.0f;
    const float vc = cj < n ? vraw * kPreScale : kSentinel;
    float sc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) sc[u] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vc), 16 * w + u));
    // row blocks J + k, k in [k0, k1], of this workgroup
    const int KJ = (B - 1) / 2 + ((B % 2 == 0 && J < B / 2) ? 1 : 0);
    const int k0 = 1 + s * ki, k1 = min(KJ, s * ki + ki);
    if (s == 0) {
        // the block's own pairs, ordered, row sums only (a cell's term with
        // itself is exactly zero); wave 0 also sums the block's voltages
        float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
        for (int u = 0; u < 16; u += 2) {
            const float d0 = vc - sc[u], d1 = vc - sc[u + 1];
            a0 = fmaf(d0, __builtin_amdgcn_exp2f(-(d0 * d0)), a0);
            a1 = fmaf(d1, __builtin_amdgcn_exp2f(-(d1 * d1)), a1);
        }
        s_row[w][kSymMaxKi][lane] = a0 + a1;
        if (w == 0) {
            double t = (double)vraw;
            for (int m = 32; m > 0; m >>= 1) t += __shfl_xor(t, m, 64);
            if (lane == 0) bsum[J] = t;
        }
    }
    float acol[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acol[u] = 0.0f;
    auto row_v = [&](int k) {
        const int i = ((J + k) % B) * 64 + lane;
        return i < n ? vd[i] * kPreScale : kSentinel;
    };
    float vnext = k0 <= k1 ? row_v(k0) : 0.0f;
    for (int k = k0; k <= k1; ++k) {
        const float vi = vnext;
        if (k < k1) vnext = row_v(k + 1);
        float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
        for (int u = 0; u < 16; u += 2) {
            const float d0 = vi - sc[u], d1 = vi - sc[u + 1];
            const float e0 = __builtin_amdgcn_exp2f(-(d0 * d0)), e1 = __builtin_amdgcn_exp2f(-(d1 * d1));
            a0 = fmaf(d0, e0, a0);
            a1 = fmaf(d1, e1, a1);
            acol[u] = fmaf(-d0, e0, acol[u]);
            acol[u + 1] = fmaf(-d1, e1, acol[u + 1]);
        }
        s_row[w][k - k0][lane] = a0 + a1;
    }
    // column sums over the 64 lanes: lane l ends with column 16w + (l & 15)'s
    sym_halve<8>(acol, lane);
    sym_halve<4>(acol, lane);
    sym_halve<2>(acol, lane);
    sym_halve<1>(acol, lane);
    float c = acol[0];
    c += __shfl_xor(c, 16, 64);
    c += __shfl_xor(c, 32, 64);
    if (lane < 16) pcol[((int64_t)J * S + s) * 64 + 16 * w + lane] = c;
    __syncthreads();
    // row sums: the four waves' parts in wave order; wave w stores rows
    // blocks k0 + w, k0 + w + 4, .. (and wave 0 the block's own)
    for (int q = w; q <= k1 - k0; q += 4)
        prow[((int64_t)((J + k0 + q) % B) * K + (k0 + q - 1)) * 64 + lane] =
            ((s_row[0][q][lane] + s_row[1][q][lane]) + s_row[2][q][lane]) + s_row[3][q][lane];
    if (s == 0 && w == 0)
        pdiag[(int64_t)J * 64 + lane] = ((s_row[0][kSymMaxKi][lane] + s_row[1][kSymMaxKi][lane]) +
                                         s_row[2][kSymMaxKi][lane]) + s_row[3][kSymMaxKi][lane];
}

// One workgroup per kVsumCells cells: thread k adds voltages k, k + 256, ..
// in fp64, the lanes combine by a fixed butterfly and the waves in wave order,
// so the step's sum of the groups' sums is the same every step. The loads
// are all issued before the first add (one memory round trip per thread).
static __global__ __launch_bounds__(256) void k_vsum(const float* __restrict__ vd, int n,
                                                     double* __restrict__ out) {
    constexpr int kPer = kVsumCells / 256;
    __shared__ double s_w[4];
    const int base = blockIdx.x * kVsumCells;
    const int m = min(kVsumCells, n - base);
    float v[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {   // past the last cell: load it again, add 0
        const int k = threadIdx.x + 256 * i;
        const float x = vd[base + min(k, m - 1)];
        v[i] = k < m ? x : 0.0f;
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) s += (double)v[i];
    for (int h = 32; h > 0; h >>= 1) s += __shfl_xor(s, h, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

template <int BLOCK>
__device__ __forceinline__ void gap_dense(const StepArgs& a, const InstDesc& d, const Tile& t,
                                          const float* __restrict__ vd, float* s_ig) {
    constexpr int W = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = d.n;
    for (int r = t.row0 + wave; r < t.row1; r += W) {
        const float vi = vd[r];
        const float* wr = a.w + d.w_off + (int64_t)r * n;
        float acc = 0.0f;
        if (d.sgj) {
            for (int j = lane; j < n; j += 64) acc = fmaf(wr[j], vi - vd[j], acc);
        } else {
            for (int j = lane; j < n; j += 64) {
                const float dv = vi - vd[j];
                acc = fmaf(wr[j], dv * gap_factor(dv), acc);
            }
        }
        acc = wave_sum_xor(acc, 64);
        if (lane == 0) s_ig[r - t.row0] = acc;
    }
}

template <int BLOCK, bool LDS, bool C16, bool HASW, bool SGJ>
__device__ __forceinline__ void gap_csr_impl(const StepArgs& a, const InstDesc& d, const Tile& t,
                                             const float* __restrict__ vd, const float* s_vd,
                                             float* s_part, float* s_ig) {
    // L lanes per row (4..BLOCK, power of two); a row wider than a wave
    // spans L/64 consecutive waves and is reduced through LDS.
    const int L = d.lanes_per_row;
    const int groups = BLOCK / L;
    const int grp = threadIdx.x / L;
    const int lig = threadIdx.x % L;
    const int64_t* rp = a.row_ptr + d.rp_off;
    const int32_t* c32 = a.col + d.w_off;
    const uint16_t* c16 = a.col16 + d.w_off;
    const float* wv = a.w + d.w_off;
    auto col_at = [&](int64_t k) -> int { return C16 ? (int)c16[k] : c32[k]; };
    // LDS: staged voltages are prescaled (gap_factor_ps), the row sum is
    // scaled back at the end
    auto v_at = [&](int j) -> float { return LDS ? s_vd[j] : vd[j]; };
    auto term = [&](float w, float vi, float vj) -> float {
        const float dv = vi - vj;
        const float f = pair_factor<SGJ, LDS>(dv);
        return HASW ? w * (dv * f) : dv * f;
    };
    const float back = LDS ? kInvPreScale : 1.0f;
    for (int r0 = t.row0; r0 < t.row1; r0 += groups) {
        const int r = r0 + grp;
        float acc0 = 0.0f, acc1 = 0.0f;
        if (r < t.row1) {
            const float vi = v_at(r);
            const int64_t e = rp[r + 1];
            int64_t k = rp[r] + lig;
            // batches of kBatch independent edges: all loads issue before use
            for (; k + (kBatch - 1) * L < e; k += kBatch * L) {
                int j[kBatch];
                float w[kBatch], v[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    j[u] = col_at(k + u * L);
                    w[u] = HASW ? wv[k + u * L] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) v[u] = v_at(j[u]);
#pragma unroll
                for (int u = 0; u < kBatch; u += 2) {
                    acc0 += term(w[u], vi, v[u]);
                    acc1 += term(w[u + 1], vi, v[u + 1]);
                }
            }
            // the remaining (< kBatch) edges of this lane as one masked
            // batch, so their loads are in flight together as well
            if (k < e) {
                int j[kBatch];
                float w[kBatch], v[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const bool ok = k + u * L < e;
                    j[u] = ok ? col_at(k + u * L) : r;      // the row itself: dV = 0
                    w[u] = HASW && ok ? wv[k + u * L] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) v[u] = v_at(j[u]);
#pragma unroll
                for (int u = 0; u < kBatch; u += 2) {
                    acc0 += term(w[u], vi, v[u]);
                    acc1 += term(w[u + 1], vi, v[u + 1]);
                }
            }
        }
        float acc = acc0 + acc1;
        if (L <= 64) {
            // all lanes of a group run the butterfly together
            acc = wave_sum_xor(acc, L) * back;
            if (r < t.row1 && lig == 0) s_ig[r - t.row0] = HASW ? acc : d.g * acc;
        } else {
            acc = wave_sum_xor(acc, 64);
            const int wave = threadIdx.x >> 6;
            if ((threadIdx.x & 63) == 0) s_part[wave] = acc;
            __syncthreads();
            if (lig == 0 && r < t.row1) {
                float tot = 0.0f;
                for (int w = 0; w < L / 64; ++w) tot += s_part[wave + w];
                tot *= back;
                s_ig[r - t.row0] = HASW ? tot : d.g * tot;
            }
            __syncthreads();
        }
    }
}

constexpr int kBlkPasses = 4;       // row passes per tile kept in registers

template <int BLOCK, bool C16, bool HASW>
__device__ __forceinline__ void gap_csr_blocked(const StepArgs& a, const InstDesc& d, const Tile& t,
                                                const float* __restrict__ vd, float* s_vd, float* s_part,
                                                float* s_ig) {
    const int L = d.lanes_per_row;
    const int groups = BLOCK / L;
    const int grp = threadIdx.x / L;
    const int lig = threadIdx.x % L;
    const int C = a.blk_cols;
    const int64_t* rp = a.row_ptr + d.rp_off;
    const int32_t* c32 = a.col + d.w_off;
    const uint16_t* c16 = a.col16 + d.w_off;
    const float* wv = a.w + d.w_off;
    const int32_t* bo = a.blk + d.blk_off;
    float acc[kBlkPasses], vi[kBlkPasses];
#pragma unroll
    for (int q = 0; q < kBlkPasses; ++q) {
        acc[q] = 0.0f;
        const int r = t.row0 + q * groups + grp;
        vi[q] = r < t.row1 ? vd[r] * kPreScale : 0.0f;
    }
    for (int b = 0; b < d.nblk; ++b) {
        const int j0 = b * C;
        const int jn = min(C, d.n - j0);
        __syncthreads();
        for (int k = threadIdx.x; k < jn; k += BLOCK) s_vd[k] = vd[j0 + k] * kPreScale;
        __syncthreads();
        const float* sb = s_vd - j0;      // indexed by the global column
#pragma unroll
        for (int q = 0; q < kBlkPasses; ++q) {
            const int r = t.row0 + q * groups + grp;
            if (r >= t.row1) continue;
            const int64_t rs = rp[r];
            const int64_t e = b + 1 < d.nblk ? rs + bo[(int64_t)r * d.nblk + b + 1] : rp[r + 1];
            int64_t k = rs + bo[(int64_t)r * d.nblk + b] + lig;
            float a0 = 0.0f, a1 = 0.0f;
            for (; k + (kBatch - 1) * L < e; k += kBatch * L) {
                int j[kBatch];
                float w[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    j[u] = C16 ? (int)c16[k + u * L] : c32[k + u * L];
                    w[u] = HASW ? wv[k + u * L] : 1.0f;
                }
#pragma unroll
                for (int u = 0; u < kBatch; u += 2) {
                    const float d0 = vi[q] - sb[j[u]], d1 = vi[q] - sb[j[u + 1]];
                    a0 = fmaf(w[u], d0 * gap_factor_ps(d0), a0);
                    a1 = fmaf(w[u + 1], d1 * gap_factor_ps(d1), a1);
                }
            }
            // the remaining (< kBatch) edges as one masked batch: loads in
            // flight together; a masked entry reads slot 0 with weight 0
            if (k < e) {
                int j[kBatch];
                float w[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const bool ok = k + u * L < e;
                    j[u] = ok ? (C16 ? (int)c16[k + u * L] : c32[k + u * L]) : j0;
                    w[u] = ok ? (HASW ? wv[k + u * L] : 1.0f) : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kBatch; u += 2) {
                    const float d0 = vi[q] - sb[j[u]], d1 = vi[q] - sb[j[u + 1]];
                    a0 = fmaf(w[u], d0 * gap_factor_ps(d0), a0);
                    a1 = fmaf(w[u + 1], d1 * gap_factor_ps(d1), a1);
                }
            }
            acc[q] += a0 + a1;
        }
    }
#pragma unroll
    for (int q = 0; q < kBlkPasses; ++q) {
        const int r = t.row0 + q * groups + grp;
        float v = acc[q];
        if (L <= 64) {
            v = wave_sum_xor(v, L) * kInvPreScale;
            if (r < t.row1 && lig == 0) s_ig[r - t.row0] = HASW ? v : d.g * v;
        } else {
            v = wave_sum_xor(v, 64);
            const int wave = threadIdx.x >> 6;
            __syncthreads();
            if ((threadIdx.x & 63) == 0) s_part[wave] = v;
            __syncthreads();
            if (lig == 0 && r < t.row1) {
                float tot = 0.0f;
                for (int w = 0; w < L / 64; ++w) tot += s_part[wave + w];
                tot *= kInvPreScale;
                s_ig[r - t.row0] = HASW ? tot : d.g * tot;
            }
        }
    }
}

// ---------------------------------------------------------------- chunked CSR
// Column lists in 16-byte chunks of eight 16-bit columns, read with one
// vector load per lane per chunk: the L lanes of a row read consecutive
// chunks, so a row's 128-byte cache line is touched by one load instruction.
// Padding entries make a zero term (their voltage is the row's own, dV = 0).
constexpr int kChunkCols = 8;

__device__ __forceinline__ uint4 pad_chunk(uint32_t v) {
    const uint32_t w = v | (v << 16);
    return make_uint4(w, w, w, w);
}

// Sixteen edges of a row from two chunks: columns j, voltages from `src`
// (LDS, prescaled; or global), accumulated into acc0/acc1.
template <bool PS, bool HASW, bool SGJ>
__device__ __forceinline__ void chunk_pair_terms(const uint4 q0, const uint4 q1, const float4* w4,
                                                 const float* src, float vi, float& acc0, float& acc1) {
    const uint32_t wd[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    float v[2 * kChunkCols];
#pragma unroll
    for (int e = 0; e < 2 * kChunkCols; ++e) {
        const uint32_t j = (e & 1) ? (wd[e >> 1] >> 16) : (wd[e >> 1] & 0xffffu);
        v[e] = src[j];
    }
#pragma unroll
    for (int e = 0; e < 2 * kChunkCols; e += 2) {
        const float d0 = vi - v[e], d1 = vi - v[e + 1];
        const float f0 = pair_factor<SGJ, PS>(d0);
        const float f1 = pair_factor<SGJ, PS>(d1);
        if (HASW) {
            const float4 wa = w4[e >> 2];
            const float w0 = (e & 3) == 0 ? wa.x : wa.z, w1 = (e & 3) == 0 ? wa.y : wa.w;
            acc0 = fmaf(w0, d0 * f0, acc0);
            acc1 = fmaf(w1, d1 * f1, acc1);
        } else {
            acc0 = fmaf(d0, f0, acc0);
            acc1 = fmaf(d1, f1, acc1);
        }
    }
}

// Gathers over whole rows (networks of at most 65,536 cells): row r's chunks
// [ca[r], ca[r + 1]), padded with r itself.
template <int BLOCK, bool LDS, bool HASW, bool SGJ>
__device__ __forceinline__ void gap_chunks(const StepArgs& a, const InstDesc& d, const Tile& t,
                                           const float* __restrict__ vd, const float* s_vd, float* s_part,
                                           float* s_ig) {
    const int L = d.lanes_per_row;
    const int groups = BLOCK / L;
    const int grp = threadIdx.x / L;
    const int lig = threadIdx.x % L;
    const int32_t* ca = a.ca + d.ca_off;
    const uint4* ch = a.chk + d.chk_off;
    const float4* cw = reinterpret_cast<const float4*>(a.chkw) + 2 * d.chk_off;
    const float* src = LDS ? s_vd : vd;
    const float back = LDS ? kInvPreScale : 1.0f;
    for (int r0 = t.row0; r0 < t.row1; r0 += groups) {
        const int r = r0 + grp;
        float acc0 = 0.0f, acc1 = 0.0f;
        if (r < t.row1) {
            const float vi = src[r];
            const uint4 padc = pad_chunk((uint32_t)r);
            const int ce = ca[r + 1];
            for (int c = ca[r] + lig; c < ce; c += 2 * L) {
                const bool ok1 = c + L < ce;
                const uint4 q0 = ch[c];
                const uint4 q1 = ok1 ? ch[c + L] : padc;
                float4 w4[4];
                if (HASW) {
                    w4[0] = cw[2 * (int64_t)c];
                    w4[1] = cw[2 * (int64_t)c + 1];
                    w4[2] = ok1 ? cw[2 * (int64_t)(c + L)] : make_float4(0.f, 0.f, 0.f, 0.f);
                    w4[3] = ok1 ? cw[2 * (int64_t)(c + L) + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
                }
                chunk_pair_terms<LDS, HASW, SGJ>(q0, q1, w4, src, vi, acc0, acc1);
            }
        }
        float acc = acc0 + acc1;
        if (L <= 64) {
            acc = wave_sum_xor(acc, L) * back;
            if (r < t.row1 && lig == 0) s_ig[r - t.row0] = HASW ? acc : d.g * acc;
        } else {
            acc = wave_sum_xor(acc, 64);
            const int wave = threadIdx.x >> 6;
            if ((threadIdx.x & 63) == 0) s_part[wave] = acc;
            __syncthreads();
            if (lig == 0 && r < t.row1) {
                float tot = 0.0f;
                for (int w = 0; w < L / 64; ++w) tot += s_part[wave + w];
                tot *= back;
                s_ig[r - t.row0] = HASW ? tot : d.g * tot;
            }
            __syncthreads();
        }
    }
}

constexpr int kSelfSlots = 256;     // LDS slots after a column block: the tile rows' own voltages

// Column blocks with chunks: per row and block, the columns relative to the
// block start, padded with S + (r mod 256), S = min(n, C), the LDS slot
// holding row r's own (prescaled) voltage; LDS holds S + kSelfSlots floats.
template <int BLOCK, bool HASW, bool SGJ>
__device__ __forceinline__ void gap_chunks_blocked(const StepArgs& a, const InstDesc& d, const Tile& t,
                                                   const float* __restrict__ vd, float* s_vd, float* s_part,
                                                   float* s_ig) {
    const int L = d.lanes_per_row;
    const int groups = BLOCK / L;
    const int grp = threadIdx.x / L;
    const int lig = threadIdx.x % L;
    const int C = a.blk_cols;
    const int64_t n1 = d.n + 1;
    const int32_t* cb = a.cb + d.cb_off;   // [nblk][n + 1]: block-major chunk starts
    const uint4* ch = a.chk + d.chkb_off;
    const float4* cw = reinterpret_cast<const float4*>(a.chkw) + 2 * d.chkb_off;
    const int S = C;               // own-voltage slots follow the block's C slots
    for (int k = threadIdx.x; k < t.row1 - t.row0; k += BLOCK)
        s_vd[S + ((t.row0 + k) & (kSelfSlots - 1))] = vd[t.row0 + k] * kPreScale;
    float acc[kBlkPasses], vi[kBlkPasses];
#pragma unroll
    for (int q = 0; q < kBlkPasses; ++q) {
        acc[q] = 0.0f;
        const int r = t.row0 + q * groups + grp;
        vi[q] = r < t.row1 ? vd[r] * kPreScale : 0.0f;
    }
    for (int b = 0; b < d.nblk; ++b) {
        const int j0 = b * C;
        const int jn = min(C, d.n - j0);
        __syncthreads();
        for (int k = threadIdx.x; k < jn; k += BLOCK) s_vd[k] = vd[j0 + k] * kPreScale;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kBlkPasses; ++q) {
            const int r = t.row0 + q * groups + grp;
            if (r >= t.row1) continue;
            const uint4 padc = pad_chunk((uint32_t)(S + (r & (kSelfSlots - 1))));
            const int ce = cb[b * n1 + r + 1];
            float a0 = 0.0f, a1 = 0.0f;
            for (int c = cb[b * n1 + r] + lig; c < ce; c += 2 * L) {
                const bool ok1 = c + L < ce;
                const uint4 q0 = ch[c];
                const uint4 q1 = ok1 ? ch[c + L] : padc;
                float4 w4[4];
                if (HASW) {
                    w4[0] = cw[2 * (int64_t)c];
                    w4[1] = cw[2 * (int64_t)c + 1];
                    w4[2] = ok1 ? cw[2 * (int64_t)(c + L)] : make_float4(0.f, 0.f, 0.f, 0.f);
                    w4[3] = ok1 ? cw[2 * (int64_t)(c + L) + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
                }
                chunk_pair_terms<true, HASW, SGJ>(q0, q1, w4, s_vd, vi[q], a0, a1);
            }
            acc[q] += a0 + a1;
        }
    }
#pragma unroll
    for (int q = 0; q < kBlkPasses; ++q) {
        const int r = t.row0 + q * groups + grp;
        float v = acc[q];
        if (L <= 64) {
            v = wave_sum_xor(v, L) * kInvPreScale;
            if (r < t.row1 && lig == 0) s_ig[r - t.row0] = HASW ? v : d.g * v;
        } else {
            v = wave_sum_xor(v, 64);
            const int wave = threadIdx.x >> 6;
            __syncthreads();
            if ((threadIdx.x & 63) == 0) s_part[wave] = v;
            __syncthreads();
            if (lig == 0 && r < t.row1) {
                float tot = 0.0f;
                for (int w = 0; w < L / 64; ++w) tot += s_part[wave + w];
                tot *= kInvPreScale;
                s_ig[r - t.row0] = HASW ? tot : d.g * tot;
            }
        }
    }
}

// ---------------------------------------------------------------- chunk stream
// Column blocks read as one flat stream per tile: in the block-major layout
// the chunks of the tile's rows in block b are one contiguous run
// [cb[b][row0], cb[b][row1]). A round is that run, cut at the network's
// round size (kStreamRound or half of it, as the tuner timed them); every
// wave takes a contiguous share of the round's 64-chunk
// sweeps (lane l the l-th chunk of a sweep: one coalesced 1 KB load), in
// pieces of kStreamSweeps sweeps. A one-byte tag per chunk (its row mod 256)
// selects the row's own voltage; the chunk's eight terms go to an LDS slot of
// their own. Waves run a round's pieces without synchronising; at the round's
// end the OWN threads owning each row (lanes of one quad) add that row's
// slots in a fixed order (bitwise reproducible). Two register sets alternate: while one piece is
// summed the next piece's loads are in flight, and the next block's voltages
// load during the current block. kStreamSets register sets rotate, so that
// the loads of kStreamSets - 1 pieces are in flight while one is summed.
constexpr int kStreamSweeps = 4;
constexpr int kStreamSets = 2;
constexpr int kStreamMaxBlocks = 8;    // column blocks whose chunk offsets a tile keeps in LDS
constexpr int kStreamCols = 16384;     // the column block (C) the stream is compiled for
constexpr int kStreamRound = 8192;     // largest round: chunk sums of two rounds fit in LDS
constexpr size_t kStaticLds = 8192;    // bound on k_step's static LDS (s_ig, s_part, s_red)

// LDS floats of a stream tile: block voltages, own voltages, chunk sums of
// two rounds, chunk offsets of every block ([nblk][kSelfSlots + 1] ints).
template <int BLOCK>
__host__ __device__ constexpr int stream_lds_floats(int C) {
    return C + kSelfSlots + 2 * kStreamRound + kStreamMaxBlocks * (kSelfSlots + 1);
}
// chunks the stream may load past a round's end (the arrays carry as many
// zeroed ones): a wave's share is rounded up to whole pieces
constexpr int kStreamSlack = (1024 / 64 + kStreamSweeps) * 64;

// Byte offset 4*j of the 16-bit column j in the low or high half of w: one
// instruction (a shift reading one half-word of its operand), where the
// plain form takes an extract and a shift.
__device__ __forceinline__ uint32_t col_lo_bytes(uint32_t w) {
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(r) : "v"(w));
    return r;
}
__device__ __forceinline__ uint32_t col_hi_bytes(uint32_t w) {
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1"
        : "=v"(r) : "v"(w));
    return r;
}

// One chunk's eight terms (voltages prescaled, staged in LDS). The staged
// block is the first thing in LDS (the stream variant of k_step has no
// static LDS; the runtime checks it before it offers the stream), so a
// column's LDS address is the column times four, with no base to add.
typedef const __attribute__((address_space(3))) float lds_float;
template <bool SGJ>
__device__ __forceinline__ float chunk_terms(const uint4 q, float vi) {
    const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
    float v[kChunkCols];
#pragma unroll
    for (int e = 0; e < kChunkCols; ++e)
        v[e] = *(lds_float*)(size_t)((e & 1) ? col_hi_bytes(wd[e >> 1]) : col_lo_bytes(wd[e >> 1]));
    float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
    for (int e = 0; e < kChunkCols; e += 2) {
        const float d0 = vi - v[e], d1 = vi - v[e + 1];
        a0 = fmaf(d0, pair_factor<SGJ, true>(d0), a0);
        a1 = fmaf(d1, pair_factor<SGJ, true>(d1), a1);
    }
    return a0 + a1;
}

// One piece of a wave's share of a round: block b (whose run ends at re),
// round [r0, r1), the wave's first sweep s0 and its sweeps in this piece np
// (0..kStreamSweeps), the piece's index in the share and the pieces per
// share; b == nblk: none.
struct StreamPiece {
    int b, re, r0, r1, s0, np, j, npieces;
};

template <int BLOCK, bool SGJ>
__device__ __forceinline__ void gap_stream_blocked(const StepArgs& a, const InstDesc& d, const Tile& t,
                                                   const float* __restrict__ vd, float* s_vd, float* s_ig) {
    constexpr int W = BLOCK / 64;
    constexpr int OWN = BLOCK / kSelfSlots;               // threads owning one row
    constexpr int STAGE = kStreamCols / BLOCK;            // block voltages staged per thread (C = kStreamCols)
    constexpr int SW = kStreamSweeps;
    static_assert(OWN >= 1 && OWN <= 64, "owners per row");
    // chunks per round: the descriptor's (the tuner times kStreamRound and
    // half of it), else kStreamRound; the LDS holds two rounds of kStreamRound
    const int RND = (d.stream_round >= 64 && d.stream_round <= kStreamRound) ? d.stream_round : kStreamRound;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // descriptor fields in registers: read once, not again inside the loop
    // (a load there would wait for the chunk loads in flight)
    const int C = kStreamCols;
    const int n = d.n;
    const int nblk = d.nblk;
    const float g = d.g;
    float* s_self = s_vd + C;                   // row r's own voltage at C + (r mod 256)
    float* s_sums = s_self + kSelfSlots;        // per-chunk sums of a round, rounds alternating buffers
    int* s_off = reinterpret_cast<int*>(s_sums + 2 * kStreamRound);   // [b][i]: chunk start of row row0 + i
    const int64_t n1 = n + 1;
    const int32_t* cb = a.cb + d.cb_off;
    const uint4* ch = a.chk + d.chkb_off;
    const uint8_t* tag = a.rtag + d.chkb_off;
    const int nrows = t.row1 - t.row0;
    const int nr1 = nrows + 1;
    // the tables' loads first (so that storing them waits for them only)
    constexpr int TBL = (kStreamMaxBlocks * (kSelfSlots + 1) + BLOCK - 1) / BLOCK;
    const int ntab = nblk * nr1;
    const float selfv = vd[t.row0 + min((int)threadIdx.x, nrows - 1)];
    int offv[TBL];
#pragma unroll
    for (int u = 0; u < TBL; ++u) {
        const int k = min((int)threadIdx.x + u * BLOCK, ntab - 1);
        const int b = k / nr1, i = k - b * nr1;
        offv[u] = cb[b * n1 + t.row0 + i];
    }
    const int orow = threadIdx.x / OWN, oq = threadIdx.x % OWN;
    const bool owner = orow < nrows;
    float rowacc = 0.0f;

    // Piece bounds are the same in every lane of a wave (made scalar, so that
    // branches on them are scalar: the loads and stores of the pipeline stay
    // in straight-line code and wait only for what they use).
    auto uni = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
    auto piece_of = [&](int b, int re, int r0, int r1, int j) {
        const int nsw = (r1 - r0 + 63) / 64;                 // sweeps of the round
        const int q = (nsw + W - 1) / W;                     // sweeps per wave
        const int s0 = min(nsw, wave * q + j * SW);
        const int np = min(SW, min(nsw, wave * q + q) - s0);
        return StreamPiece{b, re, r0, r1, s0, max(np, 0), j, (q + SW - 1) / SW};
    };
    auto first_round_from = [&](int b0) {    // the first piece of the first round of block b0 or later
        for (int b = b0; b < nblk; ++b) {
            const int r0 = uni(s_off[b * nr1]), re = uni(s_off[b * nr1 + nrows]);
            if (r0 < re) return piece_of(b, re, r0, min(re, r0 + RND), 0);
        }
        return StreamPiece{nblk, 0, 0, 0, 0, 0, 0, 1};
    };
    // within a block from registers only; LDS is read at block changes
    auto next_piece = [&](const StreamPiece& p) {
        if (p.j + 1 < p.npieces) return piece_of(p.b, p.re, p.r0, p.r1, p.j + 1);
        if (p.r1 < p.re) return piece_of(p.b, p.re, p.r1, min(p.re, p.r1 + RND), 0);
        return first_round_from(p.b + 1);
    };
    auto next_block = [&](int b) {     // the next block with chunks after b, nblk if none
        for (++b; b < nblk; ++b)
            if (uni(s_off[b * nr1]) < uni(s_off[b * nr1 + nrows])) return b;
        return nblk;
    };
    // every sweep slot of a piece loads (past its end, chunks the compute
    // skips: the arrays carry kStreamSlack chunks of slack), from one address
    auto load = [&](uint4 (&q)[SW], uint32_t (&tg)[SW], const StreamPiece& p) {
        const int c0 = p.r0 + p.s0 * 64 + lane;
        const uint4* qp = ch + c0;
        const uint8_t* tp = tag + c0;
#pragma unroll
        for (int i = 0; i < SW; ++i) {
            q[i] = qp[i * 64];
            tg[i] = tp[i * 64];
        }
    };
    auto compute = [&](const uint4 (&q)[SW], const uint32_t (&tg)[SW], const StreamPiece& p, float* sums) {
        const int slot = p.s0 * 64 + lane;                  // this lane's slot of sweep 0
        const int m = p.r1 - p.r0;
        float* dst = sums + slot;
        if (p.np == SW && (p.s0 + SW) * 64 <= m) {
            // whole sweeps only (all but a round's last piece): one basic
            // block, in which the scheduler overlaps two sweeps at a time
#pragma unroll
            for (int i = 0; i < SW; ++i) {
                dst[i * 64] = chunk_terms<SGJ>(q[i], s_self[tg[i]]);
                if (i & 1) __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int i = 0; i < SW; ++i) {
                if (i < p.np) {
                    const float sum = chunk_terms<SGJ>(q[i], s_self[tg[i]]);
                    if (slot + i * 64 < m) dst[i * 64] = sum;
                }
            }
        }
    };
    auto combine = [&](const StreamPiece& p, const float* sums) {
        float part = 0.0f;
        if (owner) {
            const int rlo = max(s_off[p.b * nr1 + orow], p.r0), rhi = min(s_off[p.b * nr1 + orow + 1], p.r1);
            for (int c = rlo + oq; c < rhi; c += OWN) part += sums[c - p.r0];
        }
        // the OWN owners of a row are the lanes of a quad (or half of one):
        // add them through DPP, in wave_sum_xor's order, without a trip to LDS
        static_assert(OWN == 2 || OWN == 4, "owners per row");
        if constexpr (OWN == 4)
            part += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(part), 0x4E, 0xF, 0xF, false));
        part += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(part), 0xB1, 0xF, 0xF, false));
        rowacc += part;
    };
    // all C slots are loaded and stored, past the network's last cell too:
    // the state buffer holds 14 rows of at least n > C / 2 cells after Vd,
    // and no column entry names a slot past the block's end
    // (four voltages per load and store: the network's Vd row starts on a
    // 16-byte boundary, which the runtime requires of stream networks)
    constexpr int STAGE4 = STAGE / 4;
    float4 sv[STAGE4];
    auto load_voltages = [&](int b) {
        const float4* src = reinterpret_cast<const float4*>(vd + b * C) + threadIdx.x;
#pragma unroll
        for (int u = 0; u < STAGE4; ++u) sv[u] = src[u * BLOCK];
    };
    auto store_voltages = [&]() {
        float4* dst = reinterpret_cast<float4*>(s_vd) + threadIdx.x;
#pragma unroll
        for (int u = 0; u < STAGE4; ++u)
            dst[u * BLOCK] = make_float4(sv[u].x * kPreScale, sv[u].y * kPreScale, sv[u].z * kPreScale,
                                         sv[u].w * kPreScale);
    };

    constexpr int NS = kStreamSets;
    uint4 q[NS][SW];
    uint32_t tg[NS][SW];
    StreamPiece prev{-1, 0, 0, 0, 0, 0, 0, 1};   // the round summed last (combined at the next round's start)
    int staged = -1;
    // the first piece when block 0 has chunks: its loads go out before the
    // tables are stored (the bounds from global memory; else after them)
    StreamPiece cur{nblk, 0, 0, 0, 0, 0, 0, 1};
    {
        const int g0 = uni(cb[t.row0]), g1 = uni(cb[t.row1]);
        if (nblk > 0 && g0 < g1) {
            cur = piece_of(0, g1, g0, min(g1, g0 + RND), 0);
            load_voltages(0);
            load(q[0], tg[0], cur);
        }
    }
    if (threadIdx.x < nrows) s_self[(t.row0 + threadIdx.x) & (kSelfSlots - 1)] = selfv * kPreScale;
#pragma unroll
    for (int u = 0; u < TBL; ++u)
        if ((int)threadIdx.x + u * BLOCK < ntab) s_off[threadIdx.x + u * BLOCK] = offv[u];
    __syncthreads();
    if (cur.b >= nblk) {
        cur = first_round_from(1);
        if (cur.b < nblk) {
            load_voltages(cur.b);
            load(q[0], tg[0], cur);
        }
    }
    StreamPiece ahead = cur;                     // the last piece whose loads are queued
#pragma unroll
    for (int k = 1; k < NS - 1; ++k) {
        const StreamPiece nx = ahead.b < nblk ? next_piece(ahead) : ahead;
        ahead = nx;
        if (ahead.b < nblk) load(q[k], tg[k], ahead);
    }
    int rb = 0;                                  // the sums buffer of the current round
    // Sum the piece in set u while set u - 1 (summed last) loads the piece
    // NS - 1 ahead. Every wave has the same pieces per round, so the barriers
    // at round starts match. Rounds alternate between two sums buffers: the
    // previous round's rows are added while the next block is staged.
    auto step = [&](uint4 (&qx)[SW], uint32_t (&tx)[SW], uint4 (&qz)[SW], uint32_t (&tz)[SW]) {
        if (ahead.b < nblk) {
            ahead = next_piece(ahead);
            if (ahead.b < nblk) load(qz, tz, ahead);
        }
        if (cur.j == 0) {
            __syncthreads();                    // the previous round is summed; its voltages are done with
            if (prev.b >= 0) {
                rb ^= 1;
                combine(prev, s_sums + (rb ^ 1) * kStreamRound);
            }
            if (staged != cur.b) {
                store_voltages();
                staged = cur.b;
                __syncthreads();                // the voltages are staged; the previous round's rows added
                const int nb = next_block(cur.b);   // its voltages load during this block
                if (nb < nblk) load_voltages(nb);
            }
        }
        compute(qx, tx, cur, s_sums + rb * kStreamRound);
        prev = cur;
        cur = next_piece(cur);
    };
    while (cur.b < nblk) {
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            if (cur.b < nblk) step(q[u], tg[u], q[(u + NS - 1) % NS], tg[(u + NS - 1) % NS]);
        }
    }
    __syncthreads();
    if (prev.b >= 0) combine(prev, s_sums + rb * kStreamRound);
    if (owner && oq == 0) s_ig[orow] = g * rowacc * kInvPreScale;
}

// f(std::true_type) for a network with per-edge weights when the launch
// compiles those paths (W), else f(std::false_type).
template <bool W, typename F>
__device__ __forceinline__ void by_weights(const InstDesc& d, F&& f) {
    if constexpr (W) {
        if (d.has_w) {
            f(std::true_type{});
            return;
        }
    }
    f(std::false_type{});
}

// CSR paths of one gap form (SGJ: simplified). The old column-blocked
// gathers (no chunked copy of the lists) exist for the realistic form only;
// a simplified network without chunks takes the plain gathers.
template <int BLOCK, bool SGJ, bool W>
__device__ __forceinline__ void gap_csr_form(const StepArgs& a, const InstDesc& d, const Tile& t,
                                             const float* __restrict__ vd, float* s_vd, float* s_part,
                                             float* s_ig) {
    // column-blocked tiles run in the wide launch group only (512- or
    // 1024-thread workgroups; the runtime places them there); elsewhere the
    // same rows take the gathers below
    if constexpr (BLOCK >= 512) {
        if (d.blocked && d.cb_off >= 0) {
            by_weights<W>(d, [&](auto hw) {
                gap_chunks_blocked<BLOCK, decltype(hw)::value, SGJ>(a, d, t, vd, s_vd, s_part, s_ig);
            });
            return;
        }
        if constexpr (!SGJ) {
            if (d.blocked) {
                by_weights<W>(d, [&](auto hw) {
                    if (d.col16) gap_csr_blocked<BLOCK, true, decltype(hw)::value>(a, d, t, vd, s_vd, s_part, s_ig);
                    else gap_csr_blocked<BLOCK, false, decltype(hw)::value>(a, d, t, vd, s_vd, s_part, s_ig);
                });
                return;
            }
        }
    }
    if (d.vd_lds) {
        for (int k = threadIdx.x; k < d.n; k += BLOCK) s_vd[k] = vd[k] * kPreScale;
        __syncthreads();
    }
    by_weights<W>(d, [&](auto hw) {
        constexpr bool HW = decltype(hw)::value;
        if (d.chunked && d.ca_off >= 0) {
            if (d.vd_lds) gap_chunks<BLOCK, true, HW, SGJ>(a, d, t, vd, s_vd, s_part, s_ig);
            else gap_chunks<BLOCK, false, HW, SGJ>(a, d, t, vd, s_vd, s_part, s_ig);
        } else if (d.vd_lds) {
            if (d.col16) gap_csr_impl<BLOCK, true, true, HW, SGJ>(a, d, t, vd, s_vd, s_part, s_ig);
            else gap_csr_impl<BLOCK, true, false, HW, SGJ>(a, d, t, vd, s_vd, s_part, s_ig);
        } else {
            if (d.col16) gap_csr_impl<BLOCK, false, true, HW, SGJ>(a, d, t, vd, s_vd, s_part, s_ig);
            else gap_csr_impl<BLOCK, false, false, HW, SGJ>(a, d, t, vd, s_vd, s_part, s_ig);
        }
    });
}

// W: the launch may hold networks with per-edge weights (their paths are
// compiled in; they hold a batch of weights in registers).
template <int BLOCK, bool W>
__device__ __forceinline__ void gap_csr(const StepArgs& a, const InstDesc& d, const Tile& t,
                                        const float* __restrict__ vd, float* s_vd, float* s_part,
                                        float* s_ig) {
    if (d.sgj) gap_csr_form<BLOCK, true, W>(a, d, t, vd, s_vd, s_part, s_ig);
    else gap_csr_form<BLOCK, false, W>(a, d, t, vd, s_vd, s_part, s_ig);
}

// Bitmap words of a network: group gr (128 senders), row r (padded to a
// multiple of 16 rows), block p (senders gr*128 + 32p .. +31): word
// (gr * n_pad16 + r) * 4 + p, bit t = sender gr*128 + 32p + t. LDS holds a
// chunk of prescaled Vd, contiguous.
constexpr int kBitGroup = 128;
constexpr int kBitRows = 16;
constexpr int kBitChunkGroups = kChunk / kBitGroup;            // 64 groups per LDS chunk

__host__ __device__ __forceinline__ int bitmap_rows_pad(int n) { return (n + kBitRows - 1) / kBitRows * kBitRows; }

template <int BLOCK>
__device__ __forceinline__ void gap_bitmap(const StepArgs& a, const InstDesc& d, const Tile& t,
                                           const float* __restrict__ vd, float* s_v, float* s_part,
                                           float* s_ig) {
    // Lanes are senders, the tile's 16 rows are wave-uniform: row r's 64-bit
    // coupling word for 64 senders is a scalar load and masks the pair term
    // as the lane mask of one select.
    constexpr int W = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = d.n;
    const int npad = bitmap_rows_pad(n);
    const int groups = (n + kBitGroup - 1) / kBitGroup;
    const int nrows = t.row1 - t.row0;
    float vis[kBitRows];
    float acc[kBitRows];
#pragma unroll
    for (int r = 0; r < kBitRows; ++r) {
        vis[r] = r < nrows ? vd[t.row0 + r] * kPreScale : 0.0f;
        acc[r] = 0.0f;
    }
    // words of the tile's rows in group gr: 16 rows x 4 words, contiguous
    const uint32_t* bits = a.bits + d.bits_off + (int64_t)t.row0 * 4;
    for (int g0 = 0; g0 < groups; g0 += kBitChunkGroups) {
        const int gc = min(kBitChunkGroups, groups - g0);
        __syncthreads();
        for (int k = threadIdx.x; k < gc * kBitGroup; k += BLOCK) {
            const int j = g0 * kBitGroup + k;
            s_v[k] = j < n ? vd[j] * kPreScale : kSentinel;
        }
        __syncthreads();
        const int per = (gc + W - 1) / W;
        const int gb = wave * per, ge = min(gc, gb + per);
        for (int gl = gb; gl < ge; ++gl) {
            // qword 2r + h: row r's senders (g0 + gl) * 128 + 64h + (0..63);
            // the bitmap is not written while a step runs, so it is read
            // through the constant address space (scalar loads)
            const auto wq = (const __attribute__((address_space(4))) uint64_t*)(
                bits + (int64_t)(g0 + gl) * npad * 4);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float vj = s_v[gl * kBitGroup + 64 * h + lane];
#pragma unroll
                for (int r = 0; r < kBitRows; ++r) {
                    const float dv = vis[r] - vj;
                    const float f = fmaf(0.8f, __builtin_amdgcn_exp2f(-(dv * dv)), 0.2f);
                    const float dm = __builtin_amdgcn_inverse_ballot_w64(wq[2 * r + h]) ? dv : 0.0f;
                    acc[r] = fmaf(dm, f, acc[r]);
                }
            }
        }
    }
    // Sum each row over the 64 lanes: four exchanges that halve the values
    // a lane holds (a lane with bit b of its index set keeps the upper half)
    // leave lane l with row (l & 15) summed over its 16-lane group; two
    // more add the four groups.
    float v8[8], v4[4], v2[2];
    {
        const bool up = lane & 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float keep = up ? acc[i + 8] : acc[i], send = up ? acc[i] : acc[i + 8];
            v8[i] = keep + __shfl_xor(send, 8, 64);
        }
    }
    {
        const bool up = lane & 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float keep = up ? v8[i + 4] : v8[i], send = up ? v8[i] : v8[i + 4];
            v4[i] = keep + __shfl_xor(send, 4, 64);
        }
    }
    {
        const bool up = lane & 2;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float keep = up ? v4[i + 2] : v4[i], send = up ? v4[i] : v4[i + 2];
            v2[i] = keep + __shfl_xor(send, 2, 64);
        }
    }
    float v1;
    {
        const bool up = lane & 1;
        const float keep = up ? v2[1] : v2[0], send = up ? v2[0] : v2[1];
        v1 = keep + __shfl_xor(send, 1, 64);
    }
    v1 += __shfl_xor(v1, 16, 64);
    v1 += __shfl_xor(v1, 32, 64);
    if (lane < kBitRows) s_part[wave * kBitRows + lane] = v1;
    __syncthreads();
    if (threadIdx.x < kBitRows && t.row0 + (int)threadIdx.x < t.row1) {
        float tot = 0.0f;
        for (int w = 0; w < W; ++w) tot += s_part[w * kBitRows + threadIdx.x];
        s_ig[threadIdx.x] = d.g * (tot * kInvPreScale);
    }
}

__device__ __forceinline__ float evoked_input(const StepArgs& a, const InstDesc& d, int64_t step,
                                              int li, int64_t cell) {
    float iapp = a.bias[cell];
    for (int k = 0; k < d.n_pulses; ++k) {
        const DevPulse pl = a.pulses[d.pulse_off + k];
        if (step >= pl.n0 && step < pl.n1 && li >= pl.c0 && li < pl.c1) iapp += pl.amp;
    }
    if (d.stream_off >= 0 && step >= 0 && step < d.stream_steps)
        iapp += a.i_stream[d.stream_off + step * (int64_t)d.n + li];
    return iapp;
}

// Kernel variants by the tiles a launch holds. kVarAll: any tile. kVarNoGap:
// every tile belongs to a network without gap junctions (the compartment
// update alone). kVarNoW: no network has per-edge weights. The narrow
// variants are compiled without the paths they exclude and their registers
// (kVarNoW: 85 VGPRs against 124 in 256-thread workgroups), so that more
// waves per SIMD keep loads in flight. kVarStream: every tile is a chunk
// stream tile (column blocks, no per-edge weights, no per-cell parameters),
// the only gap path it compiles.
enum : int { kVarAll = 0, kVarNoGap = 1, kVarNoW = 2, kVarStream = 3 };

template <int BLOCK, int VAR>
__device__ __forceinline__ void step_body(const StepArgs& a, const float* __restrict__ xin, float* __restrict__ xout,
                                          int64_t step_arg, int32_t step_off, float* s_ig, float* s_part,
                                          double* s_red, float4* s_v4) {
    if (a.list_reset && blockIdx.x == 0 && threadIdx.x == 0) *a.list_reset = 0u;
    const Tile t = a.tiles[blockIdx.x];
    const InstDesc& d = a.inst[t.inst];
    const int64_t step = (a.d_step ? *a.d_step : step_arg) + step_off;
    const float* vd = xin + (int64_t)SV_VD * a.stride + d.cell_off;
    const int nrows = t.row1 - t.row0;

    // The compartment update of cell row0 + k: with at most 64 rows, lane k
    // of wave 0 advances its dendrite and axon and lane k of wave 1 its soma
    // (the update is Jacobi, so the parts are independent and their
    // arithmetic is cell_step's); else thread k advances the whole cell.
    // State loads are issued first so their latency overlaps the gap work.
    const bool split = nrows <= 64;
    const int k_own = split ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
    const int part = split ? (int)(threadIdx.x >> 6) : 0;   // 0: dendrite + axon (or all), 1: soma
    const bool own = k_own < nrows && part < 2 && !a.gap_only;
    const int li = t.row0 + k_own;
    const int64_t cell = d.cell_off + li;
    float x[NSV];
    float iapp = 0.0f;
    if (own) {
#pragma unroll
        for (int v = 0; v < NSV; ++v) x[v] = xin[v * a.stride + cell];
        iapp = evoked_input(a, d, step, li, cell);
    }

    if constexpr (VAR == kVarStream) {
        if (d.sgj) gap_stream_blocked<BLOCK, true>(a, d, t, vd, reinterpret_cast<float*>(s_v4), s_ig);
        else gap_stream_blocked<BLOCK, false>(a, d, t, vd, reinterpret_cast<float*>(s_v4), s_ig);
    } else if constexpr (VAR == kVarNoGap) {
        for (int k = threadIdx.x; k < nrows; k += BLOCK) s_ig[k] = 0.0f;
    } else {
        switch (d.conn) {
            case CONN_UNIFORM:
                if (d.sgj && d.sym) gap_uniform_sum<BLOCK>(a, d, t, vd, s_ig, s_red);
                else gap_uniform<BLOCK>(a, d, t, vd, s_ig, s_v4, s_part, s_red);
                break;
            case CONN_DENSE: gap_dense<BLOCK>(a, d, t, vd, s_ig); break;
            case CONN_CSR:
                if (d.bitmap) gap_bitmap<BLOCK>(a, d, t, vd, reinterpret_cast<float*>(s_v4), s_part, s_ig);
                else gap_csr<BLOCK, VAR != kVarNoW>(a, d, t, vd, reinterpret_cast<float*>(s_v4), s_part, s_ig);
                break;
            default:
                for (int k = threadIdx.x; k < nrows; k += BLOCK) s_ig[k] = 0.0f;
                break;
        }
    }
    __syncthreads();

    if (a.gap_only) {
        for (int k = threadIdx.x; k < nrows; k += BLOCK) a.igap_out[d.cell_off + t.row0 + k] = s_ig[k];
        return;
    }
    // per-cell parameters exist in the general variant only (the runtime
    // launches networks that have them with it)
    CellParams pc = d.p;
    if constexpr (VAR == kVarAll) {
        if (own) pc = cell_params_of(a, d, cell);
    }
    if (own && split) {
        float y[NSV];
        float chk = 0.0f;
        if (part == 0) {
            cell_step_dendrite(pc, x, s_ig[k_own], iapp, a.dt, y);
            cell_step_axon(pc, x, a.dt, y);
#pragma unroll
            for (int v : {SV_VD, SV_CA, SV_R, SV_S, SV_Q, SV_VA, SV_HA, SV_XA}) {
                xout[v * a.stride + cell] = y[v];
                chk += y[v];
            }
        } else {
            cell_step_soma(pc, x, a.dt, y);
#pragma unroll
            for (int v : {SV_VS, SV_K, SV_L, SV_H, SV_N, SV_X}) {
                xout[v * a.stride + cell] = y[v];
                chk += y[v];
            }
        }
        if (a.dry) return;
        if (!isfinite(chk)) atomicOr(a.flags, 1);
        if (part == 0 && a.out_slots) a.out_ring[out_slot(a, step) + cell] = y[SV_VA];
        // axon output (wave 0): upward 0 mV crossing, time interpolated within the step
        if (part == 0 && x[SV_VA] < 0.0f && y[SV_VA] >= 0.0f) {
            const int c = a.spike_count[cell];
            if (a.spike_cap > 0) {
                const float frac = (0.0f - x[SV_VA]) / (y[SV_VA] - x[SV_VA]);
                a.spike_times[cell * a.spike_cap + (c % a.spike_cap)] = ((float)step + frac) * a.dt;
            }
            a.spike_count[cell] = c + 1;
        }
    } else if (own) {
        float y[NSV];
        cell_step(pc, x, s_ig[k_own], iapp, a.dt, y);
        float chk = 0.0f;
#pragma unroll
        for (int v = 0; v < NSV; ++v) {
            xout[v * a.stride + cell] = y[v];
            chk += y[v];
        }
        if (a.dry) return;
        if (!isfinite(chk)) atomicOr(a.flags, 1);
        if (a.out_slots) a.out_ring[out_slot(a, step) + cell] = y[SV_VA];
        // axon output: upward 0 mV crossing, time interpolated within the step
        if (x[SV_VA] < 0.0f && y[SV_VA] >= 0.0f) {
            const int c = a.spike_count[cell];
            if (a.spike_cap > 0) {
                const float frac = (0.0f - x[SV_VA]) / (y[SV_VA] - x[SV_VA]);
                a.spike_times[cell * a.spike_cap + (c % a.spike_cap)] = ((float)step + frac) * a.dt;
            }
            a.spike_count[cell] = c + 1;
        }
    }
}

// The step. Vd staging in dynamic LDS, sized per launch: the largest
// all-to-all chunk (min(n, kChunk) + 8 per wave) or the largest LDS-staged
// CSR network. The chunk stream variant has no static LDS, so its staged
// voltages start at LDS address 0 (a gather's address is its column times
// four, with no base to add) and its row sums follow the stream's region.
template <int BLOCK, int VAR = kVarAll>
__global__ __launch_bounds__(BLOCK) void k_step(StepArgs a, const float* __restrict__ xin,
                                                float* __restrict__ xout, int64_t step_arg,
                                                int32_t step_off) {
    extern __shared__ float4 s_v4[];
    if constexpr (VAR == kVarStream) {
        float* s_ig = reinterpret_cast<float*>(s_v4) + stream_lds_floats<BLOCK>(kStreamCols);
        step_body<BLOCK, VAR>(a, xin, xout, step_arg, step_off, s_ig, nullptr, nullptr, s_v4);
    } else {
        __shared__ float s_ig[kMaxTileRows];
        __shared__ float s_part[BLOCK];
        __shared__ double s_red[BLOCK / 64];
        step_body<BLOCK, VAR>(a, xin, xout, step_arg, step_off, s_ig, s_part, s_red, s_v4);
    }
}

static __global__ void k_set_step(int64_t* d_step, int64_t value) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *d_step = value;
}

}  // namespace infoli
