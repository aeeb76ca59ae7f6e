// Host side of the learned surrogate: training-data generation, training
// (forward/backward/Adam kernels), macro steps with drift check and plain
// fallback, and the standalone MLP entry points used to check the kernels.
#include "context.hpp"
#include "surrogate_kernel.hpp"

#include <mutex>

using namespace infoli_rt;

namespace {

template <typename T>
T* dev_alloc(std::vector<void*>& owned, size_t n) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) fail(INFOLI_E_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed", n * sizeof(T));
    owned.push_back(p);
    return static_cast<T*>(p);
}

// Device buffers and events of one call. On every exit, normal or by a
// failure, the stream the call queues on (nullptr: the null stream) is
// drained before anything is released, so no queued kernel or copy still
// uses a buffer when it is freed.
struct Scoped {
    hipStream_t stream = nullptr;
    std::vector<void*> owned;
    std::vector<hipEvent_t> events;
    explicit Scoped(hipStream_t st = nullptr) : stream(st) {}
    hipEvent_t event() {
        hipEvent_t e = nullptr;
        HIPX(hipEventCreate(&e));
        events.push_back(e);
        return e;
    }
    ~Scoped() {
        (void)hipStreamSynchronize(stream);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (void* p : owned) (void)hipFree(p);
    }
};

NormStats norm_of(const float* n64) {
    NormStats ns;
    std::memcpy(ns.in_mean, n64, 16 * sizeof(float));
    std::memcpy(ns.in_rstd, n64 + 16, 16 * sizeof(float));
    std::memcpy(ns.out_mean, n64 + 32, 16 * sizeof(float));
    std::memcpy(ns.out_std, n64 + 48, 16 * sizeof(float));
    return ns;
}

void ensure_surrogate_buffers(infoli_ctx* c) {
    SurrogateState& s = c->surr;
    if (s.params) return;
    s.params = c->alloc<float>(kNumParams);
    s.m = c->alloc<float>(kNumParams);
    s.v = c->alloc<float>(kNumParams);
    s.grad = c->alloc<float>((size_t)kNumParams * kGradSplits);   // split-K partials
    s.wb = c->alloc<uint16_t>(kNumParams);
    s.hold = c->alloc<int32_t>(c->stride);
    s.counters = c->alloc<unsigned long long>(4);
    HIPX(hipMemset(s.hold, 0, sizeof(int32_t) * c->stride));
    HIPX(hipMemset(s.counters, 0, sizeof(unsigned long long) * 4));
    s.list = c->alloc<PlainEntry>(c->stride);
    s.list_count = c->alloc<unsigned int>(1);
    HIPX(hipMemset(s.list_count, 0, sizeof(unsigned int)));
}

void check_params(const float* p, int64_t n) {
    if (!p) fail(INFOLI_E_INVALID_ARG, "parameter array is NULL");
    if (!finite_all(p, n)) fail(INFOLI_E_INVALID_ARG, "non-finite MLP parameter");
}

void check_norm(const float* n64) {
    check_params(n64, 64);
    for (int f = 0; f < 16; ++f) {
        if (!(n64[16 + f] > 0.0f)) fail(INFOLI_E_INVALID_ARG, "input scale %d must be > 0", f);
        if (!(n64[48 + f] > 0.0f)) fail(INFOLI_E_INVALID_ARG, "output scale %d must be > 0", f);
    }
}

void upload_weights(infoli_ctx* c, const float* params) {
    SurrogateState& s = c->surr;
    HIPX(hipMemcpy(s.params, params, sizeof(float) * kNumParams, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3((kNumParams + 255) / 256), dim3(256), 0, c->stream, s.params, s.wb);
    HIPX(hipGetLastError());
    HIPX(hipStreamSynchronize(c->stream));
}

SurrArgs surr_args(infoli_ctx* c, const infoli_drift_cfg& dc, int64_t macro_index) {
    SurrArgs a;
    std::memset(&a, 0, sizeof(a));
    a.params = c->surr.params;
    a.wb = c->surr.wb;
    a.norm = norm_of(c->surr.norm);
    a.igap = c->igap;
    a.hold = c->surr.hold;
    a.counters = c->surr.counters;
    a.theta_mv = dc.theta_mv;
    a.v_max = dc.v_max;
    a.ca_max = dc.ca_max;
    a.z_max = dc.z_max;
    a.sample_every = dc.sample_every;
    a.hold_steps = dc.hold_steps;
    a.mode = dc.mode;
    a.macro_index = macro_index;
    a.list = static_cast<PlainEntry*>(c->surr.list);
    a.list_count = c->surr.list_count;
    // checked cells this macro step: (cell + macro_index) % sample_every == 0
    a.check_first = 0;
    a.n_checks = 0;
    if (dc.mode == INFOLI_SURROGATE_MLP && dc.sample_every > 0) {
        const int64_t S = dc.sample_every;
        a.check_first = (S - macro_index % S) % S;
        a.n_checks = a.check_first < c->total_cells ? (c->total_cells - 1 - a.check_first) / S + 1 : 0;
    }
    return a;
}

// One macro step: exact gap currents from the current Vd, then the
// surrogate (or held-gap plain) update of every cell.
void launch_macro(infoli_ctx* c, hipStream_t st, const infoli_drift_cfg& dc, int from, int64_t step0) {
    StepArgs g = make_args(c, false);
    g.gap_only = 1;
    g.list_reset = c->surr.list_count;
    launch_groups(c, st, g, from, step0, 0, false);
    const StepArgs a = make_args(c, false);
    const int64_t cells = c->total_cells;
    if (dc.mode == INFOLI_SURROGATE_PLAIN_HOLD) {
        hipLaunchKernelGGL(k_hold4, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, a, c->igap,
                           c->state[from], c->state[from ^ 1], step0, cells);
        return;
    }
    const SurrArgs s = surr_args(c, dc, step0 / kMacro);
    // three workgroups (twelve waves, 148 VGPRs each) per compute unit: LDS
    // holds three 42 KB weight copies (two per CU measured 1.6 % slower)
    const unsigned blocks = (unsigned)std::min<int64_t>((cells + 63) / 64, 3 * (int64_t)c->n_cu);
    hipLaunchKernelGGL(k_surrogate_step, dim3(blocks), dim3(256), 0, st, a, s, c->state[from],
                       c->state[from ^ 1], step0, cells);
    const unsigned lblocks = (unsigned)std::min<int64_t>((cells + 63) / 64, 2048);
    hipLaunchKernelGGL(k_plain_list, dim3(lblocks), dim3(kListBlock), 0, st, a, s, c->state[from],
                       c->state[from ^ 1], step0);
}

// ---------------------------------------------------------------- staging without allocation
// Largest batch of infoli_mlp_loss_grad_noalloc and the staging memory it
// needs: the bf16 weights, the split-K partial gradients, the six transposed
// activation buffers and the per-wave loss sums, each start 256-byte aligned.
constexpr int32_t kNoAllocMaxBatch = 8192;

constexpr size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr size_t staging_bytes(int32_t batch) {
    return round256(sizeof(uint16_t) * kNumParams) + round256(sizeof(float) * kNumParams * kGradSplits) +
           2 * round256(sizeof(uint16_t) * 16 * (size_t)batch) + 4 * round256(sizeof(uint16_t) * kHid * (size_t)batch) +
           round256(sizeof(float) * (size_t)(batch / 16));
}

constexpr size_t kScratchBytes = staging_bytes(kNoAllocMaxBatch);     // 10,284,800 bytes

// Carves the staging buffers of one call out of `base` (device address).
struct Staging {
    uint16_t* wb;
    float* part;
    TrainBufs tb;
};

Staging carve(unsigned char* base, int32_t batch) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base + off;
        off += round256(bytes);
        return p;
    };
    Staging st;
    st.wb = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * kNumParams));
    st.part = reinterpret_cast<float*>(take(sizeof(float) * kNumParams * kGradSplits));
    st.tb.xT = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * 16 * (size_t)batch));
    st.tb.dyT = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * 16 * (size_t)batch));
    st.tb.h1T = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * kHid * (size_t)batch));
    st.tb.h2T = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * kHid * (size_t)batch));
    st.tb.dz2T = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * kHid * (size_t)batch));
    st.tb.dz1T = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * kHid * (size_t)batch));
    st.tb.loss_part = reinterpret_cast<float*>(take(sizeof(float) * (size_t)(batch / 16)));
    if (off != staging_bytes(batch) || off > kScratchBytes) fail(INFOLI_E_DEVICE, "staging layout mismatch");
    return st;
}

}  // namespace

// Staging memory of infoli_mlp_loss_grad_noalloc: one copy on each GPU the
// library runs on, held until the process ends. Host code never uses this
// name as an address (on the host it names a stand-in): the device address
// comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_addr[64] = {};     // per device ordinal; nullptr until looked up

// Device address of `scratch` on the current device, looked up on the first
// call there with that device current.
unsigned char* scratch_on_current_device() {
    int dev = -1;
    HIPX(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) fail(INFOLI_E_DEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(INFOLI_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_addr[dev] = p;
    }
    return static_cast<unsigned char*>(g_scratch_addr[dev]);
}

// A caller's pointer must be device memory of the current device (a host
// pointer would fault the kernels instead of failing here).
void check_device_ptr(const void* p, int dev, const char* what) {
    if (!p) fail(INFOLI_E_INVALID_ARG, "%s is NULL", what);
    hipPointerAttribute_t at{};
    const hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();            // leave no error for the next call to report
        fail(INFOLI_E_INVALID_ARG, "%s is not device memory", what);
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        fail(INFOLI_E_INVALID_ARG, "%s is not device memory", what);
    if (at.device != dev) fail(INFOLI_E_INVALID_ARG, "%s is on device %d, not the current device %d", what, at.device, dev);
}

}  // namespace

extern "C" {

infoli_status infoli_default_train_cfg(infoli_train_cfg* cfg) {
    if (!cfg) {
        g_thread_error = "cfg is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n_transitions = 1000000;
    cfg->n_trajectories = 4096;
    cfg->burn_in = 2500;
    cfg->batch = 4096;
    cfg->steps = 20000;
    cfg->lr = 1e-3f;
    cfg->lr_min = 1e-5f;
    cfg->v_max = -40.0f;
    cfg->ca_max = 20.0f;
    cfg->beta1 = 0.9f;
    cfg->beta2 = 0.999f;
    cfg->eps = 1e-8f;
    cfg->bias_sd = 0.7f;
    cfg->gap_sd = 1.5f;
    cfg->gap_rho = 0.9f;
    cfg->pulse_p = 0.005f;
    cfg->pulse_lo = 2.0f;
    cfg->pulse_hi = 8.0f;
    cfg->pulse_len = 25;
    cfg->seed = 5001;
    cfg->init_params = nullptr;
    return INFOLI_OK;
}

infoli_status infoli_default_drift_cfg(infoli_drift_cfg* cfg) {
    if (!cfg) {
        g_thread_error = "cfg is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->theta_mv = 0.5f;
    cfg->v_max = -40.0f;
    cfg->ca_max = 20.0f;
    cfg->sample_every = 64;
    cfg->hold_steps = 50;
    cfg->mode = INFOLI_SURROGATE_MLP;
    cfg->z_max = 8.0f;
    return INFOLI_OK;
}

infoli_status infoli_surrogate_train(infoli_ctx* ctx, const infoli_train_cfg* cfg, infoli_train_report* rep,
                                     float* loss_hist) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        if (!cfg) fail(INFOLI_E_INVALID_ARG, "cfg is NULL");
        if (ctx->n_inst != 1) fail(INFOLI_E_UNSUPPORTED, "the surrogate runs on single-network contexts");
        if (ctx->inst[0].pcell)
            fail(INFOLI_E_UNSUPPORTED, "the surrogate learns one parameter set: no per-cell parameters");
        if (cfg->batch < 16 || cfg->batch % 64 != 0 || cfg->batch > (1 << 20))
            fail(INFOLI_E_INVALID_ARG, "batch must be a positive multiple of 64 up to 2^20");
        if (cfg->steps < 0 || cfg->n_trajectories < 1 || cfg->n_transitions < cfg->batch ||
            cfg->burn_in < 0 || cfg->pulse_len < 0 || !(cfg->lr > 0.0f) ||
            !(cfg->lr_min >= 0.0f) || !(cfg->lr_min <= cfg->lr) ||
            !(cfg->v_max >= -50.0f && cfg->v_max < 1000.0f) || std::isnan(cfg->ca_max) ||
            !(cfg->gap_rho >= 0.0f && cfg->gap_rho < 1.0f))
            fail(INFOLI_E_INVALID_ARG, "bad training configuration");
        check_params(cfg->init_params, kNumParams);
        const int64_t per_traj = (cfg->n_transitions + cfg->n_trajectories - 1) / cfg->n_trajectories;
        const int64_t n_data = per_traj * cfg->n_trajectories;
        if (n_data > (int64_t)1 << 28) fail(INFOLI_E_INVALID_ARG, "training set too large");
        ensure_surrogate_buffers(ctx);
        SurrogateState& s = ctx->surr;
        hipStream_t st = ctx->stream;
        Scoped tmp(st);
        float* xd = dev_alloc<float>(tmp.owned, (size_t)n_data * 16);
        float* td = dev_alloc<float>(tmp.owned, (size_t)n_data * 16);
        double* stats = dev_alloc<double>(tmp.owned, 64);
        hipEvent_t e0 = tmp.event(), e1 = tmp.event(), e2 = tmp.event();
        HIPX(hipEventRecord(e0, st));

        // 1. transitions of the plain method under random currents
        DataGenArgs g;
        std::memset(&g, 0, sizeof(g));
        g.p = ctx->inst[0].p;
        rest_state_host(reinterpret_cast<const float*>(&ctx->inst[0].p), -60.0f, g.rest);
        if (!(cfg->ca_max > g.rest[SV_CA])) fail(INFOLI_E_INVALID_ARG, "ca_max must exceed the rest [Ca]");
        g.dt = ctx->dt;
        g.bias_sd = cfg->bias_sd;
        g.gap_sd = cfg->gap_sd;
        g.gap_rho = cfg->gap_rho;
        g.pulse_p = cfg->pulse_p;
        g.pulse_lo = cfg->pulse_lo;
        g.pulse_hi = cfg->pulse_hi;
        g.pulse_len = cfg->pulse_len;
        g.v_max = cfg->v_max;
        g.ca_max = cfg->ca_max;
        g.burn_in = cfg->burn_in;
        g.per_traj = (int32_t)per_traj;
        g.n_traj = cfg->n_trajectories;
        g.seed = cfg->seed;
        g.x_raw = xd;
        g.d_raw = td;
        hipLaunchKernelGGL(k_surrogate_data, dim3((g.n_traj + 127) / 128), dim3(128), 0, st, g);
        HIPX(hipGetLastError());

        // 2. normalisation from training-set statistics
        hipLaunchKernelGGL(k_feature_stats, dim3(16), dim3(256), 0, st, xd, n_data, stats);
        hipLaunchKernelGGL(k_feature_stats, dim3(16), dim3(256), 0, st, td, n_data, stats + 32);
        HIPX(hipGetLastError());
        // the statistics kernels are done before the blocking copy reads them
        // into heap memory (no copy is left in flight into a stack frame)
        HIPX(hipStreamSynchronize(st));
        std::vector<double> hs(64);
        HIPX(hipMemcpy(hs.data(), stats, sizeof(double) * 64, hipMemcpyDeviceToHost));
        float nrm[64];
        for (int f = 0; f < 16; ++f) {
            const double sd_in = hs[2 * f + 1], sd_out = hs[32 + 2 * f + 1];
            nrm[f] = (float)hs[2 * f];
            nrm[16 + f] = (float)(sd_in > 1e-12 ? 1.0 / sd_in : 1.0);
            nrm[32 + f] = f < kTargets ? (float)hs[32 + 2 * f] : 0.0f;
            nrm[48 + f] = f < kTargets && sd_out > 1e-12 ? (float)sd_out : 1.0f;
        }
        for (int k = 0; k < 64; ++k)
            if (!std::isfinite(nrm[k])) fail(INFOLI_E_NUMERIC, "training data contain non-finite values");
        std::memcpy(s.norm, nrm, sizeof(nrm));
        const NormStats ns = norm_of(nrm);
        hipLaunchKernelGGL(k_normalize, dim3((unsigned)((n_data * 16 + 255) / 256)), dim3(256), 0, st, xd, td,
                           n_data, ns);
        HIPX(hipEventRecord(e1, st));

        // 3. Adam from the given initial weights
        upload_weights(ctx, cfg->init_params);
        HIPX(hipMemsetAsync(s.m, 0, sizeof(float) * kNumParams, st));
        HIPX(hipMemsetAsync(s.v, 0, sizeof(float) * kNumParams, st));
        const int B = cfg->batch;
        TrainBufs tb;
        tb.xT = dev_alloc<uint16_t>(tmp.owned, (size_t)16 * B);
        tb.h1T = dev_alloc<uint16_t>(tmp.owned, (size_t)kHid * B);
        tb.h2T = dev_alloc<uint16_t>(tmp.owned, (size_t)kHid * B);
        tb.dyT = dev_alloc<uint16_t>(tmp.owned, (size_t)16 * B);
        tb.dz2T = dev_alloc<uint16_t>(tmp.owned, (size_t)kHid * B);
        tb.dz1T = dev_alloc<uint16_t>(tmp.owned, (size_t)kHid * B);
        tb.loss_part = dev_alloc<float>(tmp.owned, (size_t)B / 16);
        float* dloss = dev_alloc<float>(tmp.owned, (size_t)std::max(cfg->steps, 1));
        double c1 = 1.0, c2 = 1.0;
        for (int t = 1; t <= cfg->steps; ++t) {
            hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(B / 64), dim3(256), 0, st, s.params, s.wb, xd, td, n_data, B,
                               cfg->seed | 1ull, (uint64_t)t, tb);
            hipLaunchKernelGGL(k_mlp_wgrad, dim3(kGradTiles * kGradSplits), dim3(64), 0, st, tb, B, s.grad,
                               dloss + (t - 1));
            c1 *= cfg->beta1;
            c2 *= cfg->beta2;
            // cosine decay of the learning rate from lr to lr_min
            const double frac = cfg->steps > 1 ? (double)(t - 1) / (double)(cfg->steps - 1) : 0.0;
            const float lr_t = (float)(cfg->lr_min + 0.5 * (cfg->lr - cfg->lr_min) * (1.0 + std::cos(M_PI * frac)));
            hipLaunchKernelGGL(k_adam, dim3((kNumParams + 255) / 256), dim3(256), 0, st, s.params, s.m, s.v, s.grad,
                               kGradSplits, s.wb, lr_t, cfg->beta1, cfg->beta2, cfg->eps, (float)(1.0 - c1),
                               (float)(1.0 - c2));
        }
        HIPX(hipGetLastError());
        HIPX(hipEventRecord(e2, st));
        HIPX(hipEventSynchronize(e2));
        std::vector<float> hl(std::max(cfg->steps, 1));
        if (cfg->steps > 0) HIPX(hipMemcpy(hl.data(), dloss, sizeof(float) * cfg->steps, hipMemcpyDeviceToHost));
        if (loss_hist && cfg->steps > 0) std::memcpy(loss_hist, hl.data(), sizeof(float) * cfg->steps);
        if (rep) {
            std::memset(rep, 0, sizeof(*rep));
            rep->n_transitions = n_data;
            rep->steps = cfg->steps;
            rep->loss_first = cfg->steps ? hl[0] : 0.0f;
            rep->loss_last = cfg->steps ? hl[cfg->steps - 1] : 0.0f;
            HIPX(hipEventElapsedTime(&rep->data_ms, e0, e1));
            HIPX(hipEventElapsedTime(&rep->train_ms, e1, e2));
        }
        s.ready = true;
    });
}

infoli_status infoli_surrogate_get(infoli_ctx* ctx, float* params, float* norm) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        if (!ctx->surr.ready) fail(INFOLI_E_STATE, "no surrogate trained or set");
        HIPX(hipStreamSynchronize(ctx->stream));
        if (params) HIPX(hipMemcpy(params, ctx->surr.params, sizeof(float) * kNumParams, hipMemcpyDeviceToHost));
        if (norm) std::memcpy(norm, ctx->surr.norm, sizeof(float) * 64);
    });
}

infoli_status infoli_surrogate_set(infoli_ctx* ctx, const float* params, const float* norm) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        if (ctx->n_inst != 1) fail(INFOLI_E_UNSUPPORTED, "the surrogate runs on single-network contexts");
        check_params(params, kNumParams);
        check_norm(norm);
        ensure_surrogate_buffers(ctx);
        HIPX(hipStreamSynchronize(ctx->stream));
        upload_weights(ctx, params);
        std::memcpy(ctx->surr.norm, norm, sizeof(float) * 64);
        ctx->surr.ready = true;
    });
}

infoli_status infoli_step_surrogate(infoli_ctx* ctx, int64_t n_macro, const infoli_drift_cfg* cfg,
                                    infoli_drift_report* rep) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        infoli_drift_cfg dc;
        infoli_default_drift_cfg(&dc);
        if (cfg) dc = *cfg;
        if (n_macro < 0) fail(INFOLI_E_INVALID_ARG, "n_macro must be >= 0");
        if (ctx->out_slots > 0)
            fail(INFOLI_E_INVALID_ARG, "surrogate macro steps do not write the output ring; "
                                       "use a context without output_ring_steps");
        for (int k = 0; k < ctx->n_inst; ++k)
            if (ctx->inst[k].pcell)
                fail(INFOLI_E_UNSUPPORTED, "the surrogate learns one parameter set: no per-cell parameters");
        if (dc.mode != INFOLI_SURROGATE_MLP && dc.mode != INFOLI_SURROGATE_PLAIN_HOLD)
            fail(INFOLI_E_INVALID_ARG, "unknown surrogate mode %d", dc.mode);
        if (dc.sample_every < 0 || dc.hold_steps < 0 || !(dc.theta_mv >= 0.0f) || std::isnan(dc.v_max) ||
            std::isnan(dc.ca_max) || !(dc.z_max >= 0.0f))
            fail(INFOLI_E_INVALID_ARG, "bad drift configuration");
        if (ctx->n_inst != 1) fail(INFOLI_E_UNSUPPORTED, "the surrogate runs on single-network contexts");
        ensure_surrogate_buffers(ctx);
        if (dc.mode == INFOLI_SURROGATE_MLP && !ctx->surr.ready)
            fail(INFOLI_E_STATE, "no surrogate trained or set");
        unsigned long long before[4];
        HIPX(hipStreamSynchronize(ctx->stream));
        HIPX(hipMemcpy(before, ctx->surr.counters, sizeof(before), hipMemcpyDeviceToHost));
        HIPX(hipEventRecord(ctx->ev0, ctx->stream));
        for (int64_t m = 0; m < n_macro; ++m) {
            launch_macro(ctx, ctx->stream, dc, ctx->cur, ctx->step);
            ctx->cur ^= 1;
            ctx->step += kMacro;
        }
        HIPX(hipGetLastError());
        HIPX(hipEventRecord(ctx->ev1, ctx->stream));
        ctx->timed = true;
        if (rep) {
            HIPX(hipEventSynchronize(ctx->ev1));
            unsigned long long after[4];
            HIPX(hipMemcpy(after, ctx->surr.counters, sizeof(after), hipMemcpyDeviceToHost));
            std::memset(rep, 0, sizeof(*rep));
            rep->plain_cell_macro_steps = (int64_t)(after[0] - before[0]);
            rep->checked = (int64_t)(after[1] - before[1]);
            rep->flagged = (int64_t)(after[2] - before[2]);
            rep->guarded = (int64_t)(after[3] - before[3]);
            HIPX(hipEventElapsedTime(&rep->ms, ctx->ev0, ctx->ev1));
        }
    });
}

infoli_status infoli_mlp_forward(const float* params, const float* x, int32_t batch, float* y) {
    return guarded(nullptr, [&] {
        check_params(params, kNumParams);
        if (!x || !y || batch < 16 || batch % 16 != 0) fail(INFOLI_E_INVALID_ARG, "need x, y and batch % 16 == 0");
        check_params(x, (int64_t)batch * 16);
        Scoped tmp;
        float* dp = dev_alloc<float>(tmp.owned, kNumParams);
        uint16_t* dw = dev_alloc<uint16_t>(tmp.owned, kNumParams);
        float* dx = dev_alloc<float>(tmp.owned, (size_t)batch * 16);
        float* dy = dev_alloc<float>(tmp.owned, (size_t)batch * 16);
        HIPX(hipMemcpy(dp, params, sizeof(float) * kNumParams, hipMemcpyHostToDevice));
        HIPX(hipMemcpy(dx, x, sizeof(float) * batch * 16, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_mlp_to_bf16, dim3((kNumParams + 255) / 256), dim3(256), 0, 0, dp, dw);
        hipLaunchKernelGGL(k_mlp_forward, dim3((batch + 63) / 64), dim3(256), 0, 0, dp, dw, dx, batch, dy);
        HIPX(hipGetLastError());
        HIPX(hipDeviceSynchronize());
        HIPX(hipMemcpy(y, dy, sizeof(float) * batch * 16, hipMemcpyDeviceToHost));
    });
}

infoli_status infoli_mlp_loss_grad(const float* params, const float* x, const float* t, int32_t batch, float* loss,
                                   float* grad) {
    return guarded(nullptr, [&] {
        check_params(params, kNumParams);
        if (!x || !t || !grad || batch < 16 || batch % 16 != 0 || batch > (1 << 20))
            fail(INFOLI_E_INVALID_ARG, "need x, t, grad and batch % 16 == 0");
        check_params(x, (int64_t)batch * 16);
        check_params(t, (int64_t)batch * 16);
        Scoped tmp;
        float* dp = dev_alloc<float>(tmp.owned, kNumParams);
        uint16_t* dw = dev_alloc<uint16_t>(tmp.owned, kNumParams);
        float* dx = dev_alloc<float>(tmp.owned, (size_t)batch * 16);
        float* dt = dev_alloc<float>(tmp.owned, (size_t)batch * 16);
        float* dg = dev_alloc<float>(tmp.owned, kNumParams);
        float* dpart = dev_alloc<float>(tmp.owned, (size_t)kNumParams * kGradSplits);
        float* dl = dev_alloc<float>(tmp.owned, 1);
        TrainBufs tb;
        tb.xT = dev_alloc<uint16_t>(tmp.owned, (size_t)16 * batch);
        tb.h1T = dev_alloc<uint16_t>(tmp.owned, (size_t)kHid * batch);
        tb.h2T = dev_alloc<uint16_t>(tmp.owned, (size_t)kHid * batch);
        tb.dyT = dev_alloc<uint16_t>(tmp.owned, (size_t)16 * batch);
        tb.dz2T = dev_alloc<uint16_t>(tmp.owned, (size_t)kHid * batch);
        tb.dz1T = dev_alloc<uint16_t>(tmp.owned, (size_t)kHid * batch);
        tb.loss_part = dev_alloc<float>(tmp.owned, (size_t)batch / 16);
        HIPX(hipMemcpy(dp, params, sizeof(float) * kNumParams, hipMemcpyHostToDevice));
        HIPX(hipMemcpy(dx, x, sizeof(float) * batch * 16, hipMemcpyHostToDevice));
        HIPX(hipMemcpy(dt, t, sizeof(float) * batch * 16, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_mlp_to_bf16, dim3((kNumParams + 255) / 256), dim3(256), 0, 0, dp, dw);
        hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((batch + 63) / 64), dim3(256), 0, 0, dp, dw, dx, dt, (int64_t)batch,
                           batch, 0ull, 0ull, tb);
        hipLaunchKernelGGL(k_mlp_wgrad, dim3(kGradTiles * kGradSplits), dim3(64), 0, 0, tb, batch, dpart, dl);
        hipLaunchKernelGGL(k_grad_reduce, dim3((kNumParams + 255) / 256), dim3(256), 0, 0, dpart, kGradSplits, dg);
        HIPX(hipGetLastError());
        HIPX(hipDeviceSynchronize());
        HIPX(hipMemcpy(grad, dg, sizeof(float) * kNumParams, hipMemcpyDeviceToHost));
        if (loss) HIPX(hipMemcpy(loss, dl, sizeof(float), hipMemcpyDeviceToHost));
    });
}

infoli_status infoli_mlp_adam_step(float* params, float* m, float* v, const float* grad, int64_t t, float lr,
                                   float beta1, float beta2, float eps) {
    return guarded(nullptr, [&] {
        check_params(params, kNumParams);
        check_params(m, kNumParams);
        check_params(v, kNumParams);
        check_params(grad, kNumParams);
        if (t < 1 || !(lr > 0.0f)) fail(INFOLI_E_INVALID_ARG, "t >= 1 and lr > 0 required");
        Scoped tmp;
        float* dp = dev_alloc<float>(tmp.owned, kNumParams);
        float* dm = dev_alloc<float>(tmp.owned, kNumParams);
        float* dv = dev_alloc<float>(tmp.owned, kNumParams);
        float* dg = dev_alloc<float>(tmp.owned, kNumParams);
        uint16_t* dw = dev_alloc<uint16_t>(tmp.owned, kNumParams);
        HIPX(hipMemcpy(dp, params, sizeof(float) * kNumParams, hipMemcpyHostToDevice));
        HIPX(hipMemcpy(dm, m, sizeof(float) * kNumParams, hipMemcpyHostToDevice));
        HIPX(hipMemcpy(dv, v, sizeof(float) * kNumParams, hipMemcpyHostToDevice));
        HIPX(hipMemcpy(dg, grad, sizeof(float) * kNumParams, hipMemcpyHostToDevice));
        const double c1 = 1.0 - std::pow((double)beta1, (double)t), c2 = 1.0 - std::pow((double)beta2, (double)t);
        hipLaunchKernelGGL(k_adam, dim3((kNumParams + 255) / 256), dim3(256), 0, 0, dp, dm, dv, dg, 1, dw, lr, beta1,
                           beta2, eps, (float)c1, (float)c2);
        HIPX(hipGetLastError());
        HIPX(hipDeviceSynchronize());
        HIPX(hipMemcpy(params, dp, sizeof(float) * kNumParams, hipMemcpyDeviceToHost));
        HIPX(hipMemcpy(m, dm, sizeof(float) * kNumParams, hipMemcpyDeviceToHost));
        HIPX(hipMemcpy(v, dv, sizeof(float) * kNumParams, hipMemcpyDeviceToHost));
    });
}

infoli_status infoli_mlp_loss_grad_noalloc(const float* d_params, const float* d_x, const float* d_t, int32_t batch,
                                           float* d_loss, float* d_grad, void* stream) {
    return guarded(nullptr, [&] {
        if (batch < 16 || batch % 16 != 0)
            fail(INFOLI_E_INVALID_ARG, "batch %d: need a positive multiple of 16", batch);
        if (batch > kNoAllocMaxBatch)
            fail(INFOLI_E_INVALID_ARG, "batch %d exceeds the no-allocation limit of %d", batch, kNoAllocMaxBatch);
        int dev = -1;
        HIPX(hipGetDevice(&dev));
        check_device_ptr(d_params, dev, "params");
        check_device_ptr(d_x, dev, "x");
        check_device_ptr(d_t, dev, "t");
        check_device_ptr(d_grad, dev, "grad");
        if (d_loss) check_device_ptr(d_loss, dev, "loss");
        const Staging sg = carve(scratch_on_current_device(), batch);
        const hipStream_t st = static_cast<hipStream_t>(stream);
        hipLaunchKernelGGL(k_mlp_to_bf16, dim3((kNumParams + 255) / 256), dim3(256), 0, st, d_params, sg.wb);
        hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((batch + 63) / 64), dim3(256), 0, st, d_params, sg.wb, d_x, d_t,
                           (int64_t)batch, batch, 0ull, 0ull, sg.tb);
        hipLaunchKernelGGL(k_mlp_wgrad, dim3(kGradTiles * kGradSplits), dim3(64), 0, st, sg.tb, batch, sg.part,
                           d_loss);
        hipLaunchKernelGGL(k_grad_reduce, dim3((kNumParams + 255) / 256), dim3(256), 0, st, sg.part, kGradSplits,
                           d_grad);
        HIPX(hipGetLastError());
    });
}

}  // extern "C"
