// Many steps of small networks in one launch: one workgroup owns one whole
// network (up to kPersistCells cells), keeps its cells' state in registers
// across steps and exchanges the dendritic voltages through a double buffer
// in LDS. The workgroup barrier at the end of each step is the step barrier
// of Section 2.2 (step n+1 sees only step-n voltages); no cross-workgroup
// synchronisation exists, so every workgroup always runs to completion.
// Dry runs (timing) write the final state only: no spikes, outputs or flags.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cell_model.hpp"
#include "step_kernel.hpp"

namespace infoli {

constexpr int kPersistBlock = 256;
constexpr int kPersistMaxCpt = 8;                               // cells per thread
constexpr int kPersistCells = kPersistBlock * kPersistMaxCpt;   // 2048

// kPersistCpt: cells per thread, the smallest of 1, 2, 4, 8 that covers the
// largest network of the launch.
template <int kPersistCpt>
__global__ __launch_bounds__(kPersistBlock) void k_persist(StepArgs a, const float* __restrict__ xin,
                                                           float* __restrict__ xout, int64_t step0,
                                                           int64_t n_steps) {
    __shared__ float s_vd[2][kPersistBlock * kPersistCpt];
    __shared__ double s_red[kPersistBlock / 64];
    const InstDesc& d = a.inst[blockIdx.x];
    const int n = d.n;
    const int tid = threadIdx.x;

    float x[kPersistCpt][NSV];
    float bias[kPersistCpt];
    int count[kPersistCpt];
#pragma unroll
    for (int m = 0; m < kPersistCpt; ++m) {
        const int li = tid + m * kPersistBlock;
        if (li < n) {
            const int64_t cell = d.cell_off + li;
#pragma unroll
            for (int v = 0; v < NSV; ++v) x[m][v] = xin[v * a.stride + cell];
            bias[m] = a.bias[cell];
            count[m] = a.spike_count[cell];
            s_vd[0][li] = x[m][SV_VD];
        } else {
#pragma unroll
            for (int v = 0; v < NSV; ++v) x[m][v] = 0.0f;
            bias[m] = 0.0f;
            count[m] = 0;
        }
    }
    __syncthreads();

    const int64_t* rp = a.row_ptr + d.rp_off;
    const int32_t* c32 = a.col + d.w_off;
    const uint16_t* c16 = a.col16 + d.w_off;
    const float* wv = a.w + d.w_off;
    bool bad = false;

    for (int64_t s = 0; s < n_steps; ++s) {
        const int64_t step = step0 + s;
        const float* vcur = s_vd[s & 1];
        float* vnxt = s_vd[(s + 1) & 1];
        float ig[kPersistCpt];
#pragma unroll
        for (int m = 0; m < kPersistCpt; ++m) ig[m] = 0.0f;

        // gap currents of the owned cells from the step-n voltages
        if (d.conn == CONN_UNIFORM && d.sgj) {
            // simplified gap junctions: g (n Vd_i - sum_j Vd_j), the sum in
            // fp64 in a fixed order (the workgroup's network decides the
            // branch, so every thread reaches the barriers)
            double part = 0.0;
            for (int j = tid; j < n; j += kPersistBlock) part += (double)vcur[j];
            for (int m = 32; m > 0; m >>= 1) part += __shfl_xor(part, m, 64);
            if ((tid & 63) == 0) s_red[tid >> 6] = part;
            __syncthreads();
            double tot = 0.0;
            for (int w = 0; w < kPersistBlock / 64; ++w) tot += s_red[w];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < kPersistCpt; ++m) ig[m] = d.g * (float)((double)n * (double)x[m][SV_VD] - tot);
        } else if (d.conn == CONN_UNIFORM) {
            for (int j = 0; j < n; ++j) {
                const float vj = vcur[j];
#pragma unroll
                for (int m = 0; m < kPersistCpt; ++m) {
                    const float dv = x[m][SV_VD] - vj;
                    ig[m] = fmaf(dv, gap_factor(dv), ig[m]);
                }
            }
#pragma unroll
            for (int m = 0; m < kPersistCpt; ++m) ig[m] *= d.g;
        } else if (d.conn == CONN_CSR) {
#pragma unroll
            for (int m = 0; m < kPersistCpt; ++m) {
                const int li = tid + m * kPersistBlock;
                if (li < n) {
                    float acc = 0.0f;
                    const float vi = x[m][SV_VD];
                    for (int64_t k = rp[li]; k < rp[li + 1]; ++k) {
                        const int j = d.col16 ? (int)c16[k] : c32[k];
                        const float dv = vi - vcur[j];
                        const float term = d.sgj ? dv : dv * gap_factor(dv);
                        acc += d.has_w ? wv[k] * term : term;
                    }
                    ig[m] = d.has_w ? acc : d.g * acc;
                }
            }
        } else if (d.conn == CONN_DENSE) {
#pragma unroll
            for (int m = 0; m < kPersistCpt; ++m) {
                const int li = tid + m * kPersistBlock;
                if (li < n) {
                    const float* wr = a.w + d.w_off + (int64_t)li * n;
                    float acc = 0.0f;
                    const float vi = x[m][SV_VD];
                    for (int j = 0; j < n; ++j) {
                        const float dv = vi - vcur[j];
                        acc = fmaf(wr[j], d.sgj ? dv : dv * gap_factor(dv), acc);
                    }
                    ig[m] = acc;
                }
            }
        }

        // compartments, output, next voltages
#pragma unroll
        for (int m = 0; m < kPersistCpt; ++m) {
            const int li = tid + m * kPersistBlock;
            if (li < n) {
                const int64_t cell = d.cell_off + li;
                float iapp = bias[m];
                for (int k = 0; k < d.n_pulses; ++k) {
                    const DevPulse pl = a.pulses[d.pulse_off + k];
                    if (step >= pl.n0 && step < pl.n1 && li >= pl.c0 && li < pl.c1) iapp += pl.amp;
                }
                if (d.stream_off >= 0 && step < d.stream_steps)
                    iapp += a.i_stream[d.stream_off + step * (int64_t)n + li];
                float y[NSV];
                cell_step(d.p, x[m], ig[m], iapp, a.dt, y);
                if (a.out_slots && !a.dry) a.out_ring[out_slot(a, step) + cell] = y[SV_VA];
                if (x[m][SV_VA] < 0.0f && y[SV_VA] >= 0.0f) {
                    if (a.spike_cap > 0 && !a.dry) {
                        const float frac = (0.0f - x[m][SV_VA]) / (y[SV_VA] - x[m][SV_VA]);
                        a.spike_times[cell * a.spike_cap + (count[m] % a.spike_cap)] =
                            ((float)step + frac) * a.dt;
                    }
                    count[m] += 1;
                }
#pragma unroll
                for (int v = 0; v < NSV; ++v) x[m][v] = y[v];
                vnxt[li] = y[SV_VD];
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int m = 0; m < kPersistCpt; ++m) {
        const int li = tid + m * kPersistBlock;
        if (li < n) {
            const int64_t cell = d.cell_off + li;
            float chk = 0.0f;
#pragma unroll
            for (int v = 0; v < NSV; ++v) {
                xout[v * a.stride + cell] = x[m][v];
                chk += x[m][v];
            }
            bad |= !isfinite(chk);
            if (!a.dry) a.spike_count[cell] = count[m];
        }
    }
    if (bad && !a.dry) atomicOr(a.flags, 1);
}

}  // namespace infoli
