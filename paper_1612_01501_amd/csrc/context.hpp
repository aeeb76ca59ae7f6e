// Host-side context of the library, shared by the step driver (runtime.hip)
// and the surrogate (surrogate.hip). Internal: not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/infoli.h"
#include "cell_model.hpp"
#include "mlp_kernel.hpp"
#include "step_kernel.hpp"

namespace infoli_rt {

using namespace infoli;

extern thread_local std::string g_thread_error;

extern const float kDefaultParams[INFOLI_NUM_PARAMS];
extern const char* const kStateNames[INFOLI_NUM_STATE];

struct Fail {
    infoli_status code;
    std::string msg;
};

[[noreturn]] inline void fail(infoli_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    throw Fail{code, buf};
}

#define HIPX(expr)                                                                   \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            fail(e_ == hipErrorOutOfMemory ? INFOLI_E_OUT_OF_MEMORY : INFOLI_E_DEVICE, \
                 "%s: %s", #expr, hipGetErrorString(e_));                            \
    } while (0)

inline bool finite_all(const float* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

void rest_state_host(const float* P, float v0, float* x);

struct TileGroup {
    int block = 256;
    std::vector<Tile> tiles;
    Tile* d_tiles = nullptr;
    size_t cap = 0;                 // tiles d_tiles holds (reused when the tuner re-plans)
    size_t lds = 16;                // dynamic LDS bytes of the launch
    int var = 0;                    // step kernel variant for these tiles (kVarAll, kVarNoGap)
};

struct SurrogateState {
    bool ready = false;                 // weights and normalisation present
    float* params = nullptr;            // [kNumParams] fp32 masters
    float* m = nullptr;                 // Adam moments
    float* v = nullptr;
    float* grad = nullptr;
    uint16_t* wb = nullptr;             // bf16 copies
    float norm[64] = {0};               // in_mean[16] in_rstd[16] out_mean[16] out_std[16]
    int32_t* hold = nullptr;            // [cells]
    unsigned long long* counters = nullptr;   // [4] plain, checked, flagged, guarded
    void* list = nullptr;               // [cells] cells for the plain method this macro step
    unsigned int* list_count = nullptr;
};

}  // namespace infoli_rt

using namespace infoli;
using infoli_rt::fail;

struct infoli_ctx {
    infoli_rt::SurrogateState surr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    hipStream_t side_stream = nullptr;  // second branch of captured steps
    bool fork_groups = true;            // captured steps run the two launch groups concurrently
    int n_cu = 256;                     // compute units of the device
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    infoli_options opt{};
    std::string err;

    int32_t n_inst = 0;
    std::vector<InstDesc> inst;     // host copies of the descriptors
    int64_t total_cells = 0;
    int64_t stride = 0;
    int64_t pairs_per_step = 0;
    float dt = 0.05f;
    int persist_cpt = 1;            // cells per thread of the persistent kernel
    // tiles of one step, in two launches: [0] 256-thread workgroups (edge
    // gathers, small networks), [1] the wide group, 1024- or 512-thread
    // workgroups (column blocks, wide bitmaps, large all-to-all networks, or
    // every CSR class when the tuner finds one wide launch faster); captured
    // as parallel graph branches or one after the other
    infoli_rt::TileGroup grp[2];
    std::vector<int> group_of;      // launch group of each network
    std::vector<int> rows_of;       // tile rows per network
    std::vector<double> deg_of;     // mean gap-junction degree per network
    int tuned = 0;                  // networks whose tiles came from timing runs
    int tune_cached = 0;            // networks whose tiles came from the tuning cache
    int tune_mode = -1;             // whole-step launch mode the tuner chose (-1: none)

    // device memory
    std::vector<void*> allocs;
    size_t device_bytes = 0;
    float* state[2] = {nullptr, nullptr};
    int cur = 0;
    float* igap = nullptr;
    float* bias = nullptr;
    InstDesc* d_inst = nullptr;
    DevPulse* d_pulses = nullptr;
    int64_t* d_rowptr = nullptr;
    int32_t* d_col = nullptr;
    uint16_t* d_col16 = nullptr;
    uint32_t* d_bits = nullptr;
    int32_t* d_blk = nullptr;       // blocked CSR: per-row block starts
    int32_t* d_ca = nullptr;        // chunked rows: per-row chunk starts
    int32_t* d_cb = nullptr;        // chunked blocks: per-row, per-block chunk starts
    uint4* d_chk = nullptr;         // chunks of eight 16-bit columns
    float* d_chkw = nullptr;        // per-edge weights in the chunk layout
    uint8_t* d_rtag = nullptr;      // chunked blocks: per chunk, its row mod 256
    int lds_max = 65536;            // dynamic LDS one workgroup may use (bytes)
    int blk_cols = 8192;            // blocked CSR: cells per LDS block
    float* d_w = nullptr;
    float* d_stream = nullptr;
    int32_t* d_spk_count = nullptr;
    float* d_spk_times = nullptr;
    int32_t* d_flags = nullptr;
    int64_t* d_step = nullptr;
    float* d_cparams = nullptr;     // per-cell parameters [20][stride], networks that have them
    float* d_psym = nullptr;        // partial sums of the networks whose pairs are taken once

    int64_t step = 0;               // absolute index of the next step to run
    // output streaming: Va after each step in a device ring, copied out on
    // out_stream; out_first: oldest step whose output the ring can hold
    float* out_ring = nullptr;
    int32_t out_slots = 0;
    int64_t out_first = 0;
    hipStream_t out_stream = nullptr;
    hipEvent_t out_ready = nullptr, out_done = nullptr;
    bool out_pending = false;       // a copy queued since the compute stream last waited for copies
    int64_t out_pending_begin = 0;  // smallest first step of those copies
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // by starting buffer parity
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;

    template <typename T>
    T* alloc(size_t count) {
        if (count == 0) count = 1;
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess)
            fail(INFOLI_E_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                 hipGetErrorString(e));
        allocs.push_back(p);
        device_bytes += count * sizeof(T);
        return static_cast<T*>(p);
    }

    void release() {
        for (int k = 0; k < 2; ++k)
            if (graph[k]) (void)hipGraphExecDestroy(graph[k]);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (stream) (void)hipStreamSynchronize(stream);
        if (out_stream) (void)hipStreamSynchronize(out_stream);
        for (void* p : allocs) (void)hipFree(p);
        allocs.clear();
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (side_stream) (void)hipStreamDestroy(side_stream);
        if (out_stream) (void)hipStreamSynchronize(out_stream);
        if (out_ready) (void)hipEventDestroy(out_ready);
        if (out_done) (void)hipEventDestroy(out_done);
        if (out_stream) (void)hipStreamDestroy(out_stream);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace infoli_rt {

inline void set_err(infoli_ctx* ctx, const std::string& m) {
    g_thread_error = m;
    if (ctx) ctx->err = m;
}

template <typename F>
infoli_status guarded(infoli_ctx* ctx, F&& f) {
    try {
        f();
        return INFOLI_OK;
    } catch (const Fail& e) {
        set_err(ctx, e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_err(ctx, "host allocation failed");
        return INFOLI_E_OUT_OF_MEMORY;
    } catch (...) {
        set_err(ctx, "unexpected internal error");
        return INFOLI_E_DEVICE;
    }
}

StepArgs make_args(const infoli_ctx* c, bool device_step);
void launch_tiles(infoli_ctx* c, hipStream_t st, const StepArgs& a, int block, unsigned ntiles, size_t lds,
                  int from, int64_t step_arg, int32_t off, int var = 0);
// Both tile groups of one step (sequential on st, or forked onto the side
// stream when `fork` and both groups have tiles).
void launch_groups(infoli_ctx* c, hipStream_t st, const StepArgs& a, int from, int64_t step_arg, int32_t off,
                   bool fork);
int64_t tile_count(const infoli_ctx* c);
void check_instance(const infoli_ctx* c, int32_t k);

}  // namespace infoli_rt
