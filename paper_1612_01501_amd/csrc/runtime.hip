// Host side of the C ABI declared in include/infoli.h: spec validation,
// device-resident network data (Section 2.4.3: everything the run needs is
// copied to the device once), tile planning and the step driver (one
// launch per step, or chunks of steps replayed from a HIP graph).
#include <sys/stat.h>

#include "context.hpp"
#include "persist_kernel.hpp"

namespace infoli_rt {

thread_local std::string g_thread_error;

// Default cell parameters, in the order of INFOLI_NUM_PARAMS, of the
// published three-compartment inferior-olive model.
extern const float kDefaultParams[INFOLI_NUM_PARAMS];
const float kDefaultParams[INFOLI_NUM_PARAMS] = {
    4.5f,    // g_CaH
    35.0f,   // g_KCa
    0.125f,  // g_h
    0.016f,  // g_ld
    0.68f,   // g_CaL
    150.0f,  // g_Na_s
    9.0f,    // g_Kdr_s
    5.0f,    // g_K_s
    0.016f,  // g_ls
    240.0f,  // g_Na_a
    20.0f,   // g_K_a
    0.016f,  // g_la
    0.13f,   // g_int
    0.25f,   // p1
    0.15f,   // p2
    55.0f,   // V_Na
    -75.0f,  // V_K
    120.0f,  // V_Ca
    -43.0f,  // V_h
    10.0f,   // V_L
};

extern const char* const kStateNames[INFOLI_NUM_STATE];
const char* const kStateNames[INFOLI_NUM_STATE] = {"Vd", "Ca", "r", "s", "q", "Vs", "k",
                                                   "l",  "h",  "n", "x", "Va", "ha", "xa"};

// Host copy of one rest-state computation (every voltage at v0, gates and
// [Ca2+] at their steady state there).
void rest_state_host(const float* P, float v0, float* x) {
    auto boltz = [](float v, float vh, float k) { return 1.0f / (1.0f + std::exp(-(v - vh) / k)); };
    auto rexp = [](float y, float s) { return y == 0.0f ? s : y / std::expm1(y / s); };
    const float ar = 1.7f / (1.0f + std::exp(-(v0 - 5.0f) / 13.9f));
    const float br = 0.02f * rexp(v0 + 8.5f, 5.0f);
    const float r = ar / (ar + br);
    const float icah = P[0] * r * r * (v0 - P[17]);
    const float ca = -3.0f * icah / 0.075f;
    const float as = std::min(0.00002f * ca, 0.01f);
    const float ax = 0.13f * rexp(-(v0 + 25.0f), 10.0f);
    const float bx = 1.69f * std::exp(-0.0125f * (v0 + 35.0f));
    x[SV_VD] = v0;
    x[SV_CA] = ca;
    x[SV_R] = r;
    x[SV_S] = as / (as + 0.015f);
    x[SV_Q] = boltz(v0, -80.0f, -4.0f);
    x[SV_VS] = v0;
    x[SV_K] = boltz(v0, -61.0f, 4.2f);
    x[SV_L] = boltz(v0, -85.5f, -8.5f);
    x[SV_H] = boltz(v0, -70.0f, -5.8f);
    x[SV_N] = boltz(v0, -3.0f, 10.0f);
    x[SV_X] = ax / (ax + bx);
    x[SV_VA] = v0;
    x[SV_HA] = boltz(v0, -60.0f, -5.8f);
    x[SV_XA] = ax / (ax + bx);
}

}  // namespace infoli_rt

using namespace infoli_rt;

namespace {

void validate_spec(const infoli_network_spec& s, int k) {
    if (s.n_cells < 1) fail(INFOLI_E_INVALID_ARG, "network %d: n_cells must be >= 1", k);
    if (s.n_cells > (1 << 26)) fail(INFOLI_E_INVALID_ARG, "network %d: n_cells too large", k);
    if (!(s.dt_ms > 0.0f) || !std::isfinite(s.dt_ms))
        fail(INFOLI_E_INVALID_ARG, "network %d: dt_ms must be finite and > 0", k);
    if (s.step0 < 0) fail(INFOLI_E_INVALID_ARG, "network %d: step0 must be >= 0", k);
    const int64_t n = s.n_cells;
    switch (s.conn) {
        case INFOLI_CONN_NONE: break;
        case INFOLI_CONN_UNIFORM_ALL:
            if (!std::isfinite(s.g_uniform)) fail(INFOLI_E_BAD_GRAPH, "network %d: g_uniform not finite", k);
            break;
        case INFOLI_CONN_DENSE:
            if (!s.w_dense) fail(INFOLI_E_INVALID_ARG, "network %d: DENSE needs w_dense", k);
            if (n > 46340) fail(INFOLI_E_INVALID_ARG, "network %d: dense n*n overflows", k);
            if (!finite_all(s.w_dense, n * n))
                fail(INFOLI_E_BAD_GRAPH, "network %d: non-finite dense weight", k);
            break;
        case INFOLI_CONN_CSR: {
            if (!s.row_ptr) fail(INFOLI_E_INVALID_ARG, "network %d: CSR needs row_ptr", k);
            if (s.nnz < 0) fail(INFOLI_E_INVALID_ARG, "network %d: nnz < 0", k);
            if (s.nnz > 0 && !s.col) fail(INFOLI_E_INVALID_ARG, "network %d: CSR needs col", k);
            if (s.row_ptr[0] != 0) fail(INFOLI_E_BAD_GRAPH, "network %d: row_ptr[0] != 0", k);
            for (int64_t i = 0; i < n; ++i)
                if (s.row_ptr[i + 1] < s.row_ptr[i])
                    fail(INFOLI_E_BAD_GRAPH, "network %d: row_ptr decreases at row %lld", k, (long long)i);
            if (s.row_ptr[n] != s.nnz)
                fail(INFOLI_E_BAD_GRAPH, "network %d: row_ptr[n] = %lld != nnz = %lld", k,
                     (long long)s.row_ptr[n], (long long)s.nnz);
            for (int64_t e = 0; e < s.nnz; ++e)
                if (s.col[e] < 0 || s.col[e] >= s.n_cells)
                    fail(INFOLI_E_BAD_GRAPH, "network %d: column %d out of range at edge %lld", k,
                         s.col[e], (long long)e);
            // every row strictly ascending: the column-block and chunk layouts
            // cut a row into contiguous per-block runs, and a repeated column
            // would be one bit of the coupling bitmap but two gathered terms
            for (int64_t i = 0; i < n; ++i)
                for (int64_t e = s.row_ptr[i] + 1; e < s.row_ptr[i + 1]; ++e)
                    if (s.col[e] <= s.col[e - 1])
                        fail(INFOLI_E_BAD_GRAPH,
                             "network %d: row %lld columns not strictly ascending at edge %lld (%d after %d)", k,
                             (long long)i, (long long)e, s.col[e], s.col[e - 1]);
            if (s.w_csr && !finite_all(s.w_csr, s.nnz))
                fail(INFOLI_E_BAD_GRAPH, "network %d: non-finite CSR weight", k);
            if (!s.w_csr && !std::isfinite(s.g_uniform))
                fail(INFOLI_E_BAD_GRAPH, "network %d: g_uniform not finite", k);
            break;
        }
        default: fail(INFOLI_E_INVALID_ARG, "network %d: unknown conn %d", k, s.conn);
    }
    if (s.params && !finite_all(s.params, INFOLI_NUM_PARAMS))
        fail(INFOLI_E_INVALID_ARG, "network %d: non-finite parameter", k);
    if (s.params && (s.params[13] <= 0.0f || s.params[13] >= 1.0f || s.params[14] <= 0.0f ||
                     s.params[14] >= 1.0f))
        fail(INFOLI_E_INVALID_ARG, "network %d: area ratios p1, p2 must lie in (0, 1)", k);
    if (s.cell_params) {
        if (!finite_all(s.cell_params, (int64_t)INFOLI_NUM_PARAMS * n))
            fail(INFOLI_E_INVALID_ARG, "network %d: non-finite per-cell parameter", k);
        for (int64_t i = 0; i < n; ++i) {
            const float* q = s.cell_params + i * INFOLI_NUM_PARAMS;
            if (q[13] <= 0.0f || q[13] >= 1.0f || q[14] <= 0.0f || q[14] >= 1.0f)
                fail(INFOLI_E_INVALID_ARG, "network %d: cell %lld: area ratios p1, p2 must lie in (0, 1)", k,
                     (long long)i);
        }
    }
    if (s.init_state && !finite_all(s.init_state, INFOLI_NUM_STATE * n))
        fail(INFOLI_E_INVALID_ARG, "network %d: non-finite initial state", k);
    if (s.i_bias && !finite_all(s.i_bias, n)) fail(INFOLI_E_INVALID_ARG, "network %d: non-finite bias", k);
    if (s.gap_kind != INFOLI_GAP_REALISTIC && s.gap_kind != INFOLI_GAP_SIMPLIFIED)
        fail(INFOLI_E_INVALID_ARG, "network %d: gap_kind must be 0 (realistic) or 1 (simplified)", k);
    if (s.reserved0 != 0) fail(INFOLI_E_INVALID_ARG, "network %d: reserved0 must be 0", k);
    if (s.n_pulses < 0 || s.n_pulses > INFOLI_MAX_PULSES)
        fail(INFOLI_E_INVALID_ARG, "network %d: n_pulses must be in [0, %d]", k, INFOLI_MAX_PULSES);
    if (s.n_pulses > 0 && !s.pulses) fail(INFOLI_E_INVALID_ARG, "network %d: pulses is NULL", k);
    for (int p = 0; p < s.n_pulses; ++p) {
        const infoli_pulse& q = s.pulses[p];
        const int32_t c1 = q.cell_end < 0 ? s.n_cells : q.cell_end;
        if (!std::isfinite(q.amplitude) || q.step_end < q.step_begin || q.cell_begin < 0 ||
            c1 > s.n_cells || q.cell_begin > c1)
            fail(INFOLI_E_INVALID_ARG, "network %d: pulse %d has a bad range or amplitude", k, p);
    }
    if (s.i_stream) {
        if (s.i_stream_steps <= 0) fail(INFOLI_E_INVALID_ARG, "network %d: i_stream_steps must be > 0", k);
        if (!finite_all(s.i_stream, s.i_stream_steps * n))
            fail(INFOLI_E_INVALID_ARG, "network %d: non-finite input stream", k);
    }
}

// Lanes per CSR row: at most kBatch edges per lane, so that one batch of
// independent loads covers most rows.
int pick_lanes(double mean_degree, int block) {
    int L = 4;
    while (L < block && L * kBatch < mean_degree) L *= 2;
    return L;
}

}  // namespace

void infoli_rt::launch_tiles(infoli_ctx* c, hipStream_t st, const StepArgs& a, int block, unsigned ntiles,
                             size_t lds, int from, int64_t step_arg, int32_t off, int var) {
    if (ntiles == 0) return;
    const float* xin = c->state[from];
    float* xout = c->state[from ^ 1];
    if (block == 512 && var == kVarStream)
        hipLaunchKernelGGL((k_step<512, kVarStream>), dim3(ntiles), dim3(512), lds, st, a, xin, xout, step_arg, off);
    else if (block == 1024 && var == kVarStream)
        hipLaunchKernelGGL((k_step<1024, kVarStream>), dim3(ntiles), dim3(1024), lds, st, a, xin, xout, step_arg,
                           off);
    else if (block == 512 && var == kVarNoW)
        hipLaunchKernelGGL((k_step<512, kVarNoW>), dim3(ntiles), dim3(512), lds, st, a, xin, xout, step_arg, off);
    else if (block == 512)
        hipLaunchKernelGGL((k_step<512, kVarAll>), dim3(ntiles), dim3(512), lds, st, a, xin, xout, step_arg, off);
    else if (block == 1024 && var == kVarNoW)
        hipLaunchKernelGGL((k_step<1024, kVarNoW>), dim3(ntiles), dim3(1024), lds, st, a, xin, xout, step_arg, off);
    else if (block == 1024)
        hipLaunchKernelGGL((k_step<1024, kVarAll>), dim3(ntiles), dim3(1024), lds, st, a, xin, xout, step_arg, off);
    else if (var == kVarNoGap)
        hipLaunchKernelGGL((k_step<256, kVarNoGap>), dim3(ntiles), dim3(256), lds, st, a, xin, xout, step_arg, off);
    else if (var == kVarNoW)
        hipLaunchKernelGGL((k_step<256, kVarNoW>), dim3(ntiles), dim3(256), lds, st, a, xin, xout, step_arg, off);
    else
        hipLaunchKernelGGL((k_step<256, kVarAll>), dim3(ntiles), dim3(256), lds, st, a, xin, xout, step_arg, off);
}

void infoli_rt::launch_groups(infoli_ctx* c, hipStream_t st, const StepArgs& a, int from, int64_t step_arg,
                              int32_t off, bool fork) {
    // the unordered pairs of all-to-all networks first: their step reads the sums
    for (int k = 0; k < c->n_inst; ++k) {
        const InstDesc& d = c->inst[k];
        if (!d.sym) continue;
        if (d.sgj) {
            hipLaunchKernelGGL(k_vsum, dim3((unsigned)vsum_groups(d.n)), dim3(256), 0, st,
                               c->state[from] + (int64_t)SV_VD * c->stride + d.cell_off, d.n,
                               reinterpret_cast<double*>(c->d_psym + d.psym_off));
            continue;
        }
        const int64_t groups = (int64_t)sym_blocks(d.n) * sym_shares(d.n, d.sym_ki);
        hipLaunchKernelGGL(k_pairs_sym, dim3((unsigned)groups), dim3(256), 0, st,
                           c->state[from] + (int64_t)SV_VD * c->stride + d.cell_off, d.n, d.sym_ki,
                           c->d_psym + d.psym_off);
    }
    const bool both = !c->grp[0].tiles.empty() && !c->grp[1].tiles.empty();
    if (fork && both) {
        HIPX(hipEventRecord(c->fork_ev, st));
        HIPX(hipStreamWaitEvent(c->side_stream, c->fork_ev, 0));
    }
    for (int g = 1; g >= 0; --g) {
        const TileGroup& tg = c->grp[g];
        StepArgs ag = a;
        ag.tiles = tg.d_tiles;
        hipStream_t s = (fork && both && g == 1) ? c->side_stream : st;
        launch_tiles(c, s, ag, tg.block, (unsigned)tg.tiles.size(), tg.lds, from, step_arg, off, tg.var);
    }
    if (fork && both) {
        HIPX(hipEventRecord(c->join_ev, c->side_stream));
        HIPX(hipStreamWaitEvent(st, c->join_ev, 0));
    }
}

int64_t infoli_rt::tile_count(const infoli_ctx* c) {
    return (int64_t)c->grp[0].tiles.size() + (int64_t)c->grp[1].tiles.size();
}

namespace {

size_t bitmap_lds_floats(int n) {
    const int groups = (n + kBitGroup - 1) / kBitGroup;
    return (size_t)std::min(groups, kBitChunkGroups) * kBitGroup;
}

void append_tiles(std::vector<std::pair<double, Tile>>& out, int k, int n, int rows, double deg) {
    for (int r = 0; r < n; r += rows) {
        const int r1 = std::min(n, r + rows);
        out.push_back({(r1 - r) * (deg * 8.0 + 400.0), Tile{k, r, r1, 0}});
    }
}

// Launch group of a network: the wide group (1024- or 512-thread
// workgroups) for column blocks, CSR or all-to-all networks the tuner marked
// wide, and all-to-all networks of >= 4,096 cells; 256-thread workgroups
// otherwise.
int group_for(const InstDesc& d) {
    if (d.conn == CONN_CSR && (d.blocked || d.wide)) return 1;
    if (d.conn == CONN_UNIFORM && !(d.sgj && d.sym) && (d.n >= 4096 || d.wide)) return 1;
    return 0;
}

// The chunk stream's gathers address LDS by column alone, which holds while
// its kernel variants have no static LDS (their staged block starts at LDS
// address 0); read from the compiled kernels once.
bool stream_kernels_ok() {
    static const bool ok = [] {
        hipFuncAttributes a1{}, a2{};
        if (hipFuncGetAttributes(&a1, reinterpret_cast<const void*>(&k_step<1024, kVarStream>)) != hipSuccess ||
            hipFuncGetAttributes(&a2, reinterpret_cast<const void*>(&k_step<512, kVarStream>)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return a1.sharedSizeBytes == 0 && a2.sharedSizeBytes == 0;
    }();
    return ok;
}

// The chunk stream can run with this context's column blocks.
bool stream_ok(const infoli_ctx* c) { return c->blk_cols == kStreamCols && stream_kernels_ok(); }

size_t lds_floats_for(const infoli_ctx* c, const InstDesc& d, int block) {
    if (d.conn == CONN_CSR && d.blocked && d.stream && d.cb_off >= 0)   // block, own voltages, sums, offsets
        return (size_t)(block >= 1024 ? stream_lds_floats<1024>(c->blk_cols) : stream_lds_floats<512>(c->blk_cols)) +
               kMaxTileRows;   // the row sums (no static LDS in the stream variant)
    if (d.conn == CONN_CSR && d.blocked)   // the column block, then the tile rows' own voltages
        return d.cb_off >= 0 ? (size_t)c->blk_cols + kSelfSlots : (size_t)std::min(d.n, c->blk_cols);
    if (d.conn == CONN_UNIFORM && d.sgj && d.sym) return 4;
    if (d.conn == CONN_UNIFORM) return (size_t)std::min(d.n, kChunk) + 8 * (size_t)(block / 64);
    if (d.conn == CONN_CSR && d.bitmap) return bitmap_lds_floats(d.n);
    if (d.conn == CONN_CSR && d.vd_lds) return (size_t)d.n;
    return 4;
}

// Tiles of every network in their launch group, longest (estimated issue
// slots) first; dynamic LDS per group; descriptors and tiles to the device.
void finalize_tiles(infoli_ctx* c) {
    std::vector<std::pair<double, Tile>> planned[2];
    size_t floats[2] = {4, 4};
    c->group_of.assign(c->n_inst, 0);
    // the chunk stream runs in a launch of stream tiles only (its kernel
    // variant compiles no other path): a stream network that would share its
    // launch with other tiles, or has weights or per-cell parameters, takes
    // the chunked column blocks instead
    {
        bool mixed[2] = {false, false};
        for (int k = 0; k < c->n_inst; ++k) {
            const InstDesc& d = c->inst[k];
            const bool st = d.conn == CONN_CSR && d.blocked && d.stream && d.cb_off >= 0 && !d.has_w && !d.pcell &&
                            d.nblk <= kStreamMaxBlocks && d.cell_off % 4 == 0 && stream_ok(c);
            if (!st) mixed[group_for(d)] = true;
        }
        for (int k = 0; k < c->n_inst; ++k) {
            InstDesc& d = c->inst[k];
            if (d.stream && (mixed[group_for(d)] || d.has_w || d.pcell || d.cb_off < 0 || !d.blocked ||
                             d.nblk > kStreamMaxBlocks || d.cell_off % 4 != 0 || !stream_ok(c)))
                d.stream = 0;
        }
    }
    for (int k = 0; k < c->n_inst; ++k) {
        const InstDesc& d = c->inst[k];
        const int g = group_for(d);
        c->group_of[k] = g;
        int rows = c->rows_of[k];
        if (d.conn == CONN_CSR && d.blocked && d.stream && d.cb_off >= 0)   // one owner group per row
            rows = std::min(rows, kSelfSlots);
        else if (d.conn == CONN_CSR && d.blocked)   // rows the column-blocked passes of this workgroup size cover
            rows = std::min(rows, kBlkPasses * std::max(1, c->grp[g].block / std::max(1, d.lanes_per_row)));
        append_tiles(planned[g], k, d.n, rows, c->deg_of[k]);
        floats[g] = std::max(floats[g], lds_floats_for(c, d, c->grp[g].block));
    }
    for (int g = 0; g < 2; ++g) {
        TileGroup& tg = c->grp[g];
        tg.lds = ((floats[g] + 3) / 4) * sizeof(float4);
        std::stable_sort(planned[g].begin(), planned[g].end(),
                         [](const auto& x, const auto& y) { return x.first > y.first; });
        tg.tiles.clear();
        bool nogap = true, now = true, stream = !planned[g].empty();
        for (const auto& pt : planned[g]) {
            tg.tiles.push_back(pt.second);
            const InstDesc& d = c->inst[pt.second.inst];
            if (d.conn != CONN_NONE || d.pcell) nogap = false;
            if (d.has_w || d.pcell) now = false;
            if (!d.stream) stream = false;
        }
        tg.var = nogap ? kVarNoGap : stream && tg.block >= 512 ? kVarStream : now ? kVarNoW : kVarAll;
        if (tg.tiles.size() > (size_t)INT32_MAX / 2) fail(INFOLI_E_INVALID_ARG, "too many tiles");
        if (!tg.tiles.empty()) {
            if (tg.tiles.size() > tg.cap) {
                tg.d_tiles = c->alloc<Tile>(tg.tiles.size());
                tg.cap = tg.tiles.size();
            }
            HIPX(hipMemcpy(tg.d_tiles, tg.tiles.data(), sizeof(Tile) * tg.tiles.size(), hipMemcpyHostToDevice));
        }
    }
    HIPX(hipMemcpy(c->d_inst, c->inst.data(), sizeof(InstDesc) * c->n_inst, hipMemcpyHostToDevice));
}

// Coupling bitmaps of CSR networks with one weight g and the realistic gap
// form (the pattern as one bit per pair), for networks of at most 16,384
// cells while the bitmaps take at most 1 GiB together; the tuner decides
// whether the step uses them.
void build_bitmaps(infoli_ctx* c, const infoli_network_spec* specs) {
    int64_t words = 0;
    for (int k = 0; k < c->n_inst; ++k) {
        InstDesc& d = c->inst[k];
        d.bits_off = -1;
        if (d.conn != CONN_CSR || d.has_w || d.sgj || d.n > 16384 || specs[k].nnz == 0) continue;
        const int64_t groups = (d.n + kBitGroup - 1) / kBitGroup;
        const int64_t w = groups * bitmap_rows_pad(d.n) * 4;
        if ((words + w) * 4 > ((int64_t)1 << 30)) continue;
        d.bits_off = words;
        words += w;
    }
    if (words == 0) return;
    std::vector<uint32_t> h((size_t)words, 0u);
    for (int k = 0; k < c->n_inst; ++k) {
        const InstDesc& d = c->inst[k];
        if (d.bits_off < 0) continue;
        const int npad = bitmap_rows_pad(d.n);
        const infoli_network_spec& s = specs[k];
        for (int i = 0; i < d.n; ++i)
            for (int64_t e = s.row_ptr[i]; e < s.row_ptr[i + 1]; ++e) {
                const int j = s.col[e];
                const int64_t g = j / kBitGroup, p = (j % kBitGroup) / 32, t = j % 32;
                h[(size_t)(d.bits_off + (g * npad + i) * 4 + p)] |= 1u << t;
            }
    }
    c->d_bits = c->alloc<uint32_t>((size_t)words);
    HIPX(hipMemcpy(c->d_bits, h.data(), sizeof(uint32_t) * words, hipMemcpyHostToDevice));
}

// Column blocks of CSR networks too large for one LDS copy of Vd: for each
// row, the offset (from the row start) of its first edge in each block of
// blk_cols cells (columns are sorted).
void build_blocks(infoli_ctx* c, const infoli_network_spec* specs) {
    int64_t total = 0;
    for (int k = 0; k < c->n_inst; ++k) {
        InstDesc& d = c->inst[k];
        d.blk_off = -1;
        d.nblk = 0;
        if (d.conn != CONN_CSR || d.n <= kChunk || specs[k].nnz == 0) continue;
        d.nblk = (d.n + c->blk_cols - 1) / c->blk_cols;
        d.blk_off = total;
        total += (int64_t)d.n * d.nblk;
    }
    if (total == 0) return;
    std::vector<int32_t> h((size_t)total);
    for (int k = 0; k < c->n_inst; ++k) {
        const InstDesc& d = c->inst[k];
        if (d.blk_off < 0) continue;
        const infoli_network_spec& s = specs[k];
        for (int i = 0; i < d.n; ++i) {
            const int64_t rs = s.row_ptr[i], re = s.row_ptr[i + 1];
            int64_t e = rs;
            for (int b = 0; b < d.nblk; ++b) {
                while (e < re && s.col[e] < b * c->blk_cols) ++e;
                h[(size_t)(d.blk_off + (int64_t)i * d.nblk + b)] = (int32_t)(e - rs);
            }
        }
    }
    c->d_blk = c->alloc<int32_t>((size_t)total);
    HIPX(hipMemcpy(c->d_blk, h.data(), sizeof(int32_t) * total, hipMemcpyHostToDevice));
}

// Chunked column lists for 16-byte vector loads (kChunkCols 16-bit columns
// per chunk). Rows layout, for networks whose columns fit 16 bits: row i's
// columns padded with i itself to whole chunks; per row its first chunk
// ([n + 1], relative to the network's first chunk). Blocks layout, for
// networks with column blocks: per row and block of C columns, the columns
// relative to the block start padded with C + (i mod kSelfSlots) to whole
// chunks; per row and block the first chunk ([n][nblk + 1]). Per-edge
// weights follow the same layout, 0 on padding.
// A simplified all-to-all network whose voltage sum k_vsum takes once per
// step (tiled steps; by default a context's only network, from kSgjSumCells
// cells on); its tiles take a row per thread.
bool sum_once(const infoli_ctx* c, const InstDesc& d) {
    const bool want = c->opt.pair_path == 2 || (c->opt.pair_path == 0 && d.n >= kSgjSumCells && c->n_inst == 1);
    return d.conn == CONN_UNIFORM && d.sgj && want && c->opt.step_mode != INFOLI_MODE_PERSISTENT;
}

// All-to-all networks whose pairs are taken once (k_pairs_sym): the
// realistic gap term, tiled steps; by default a context's only network, from
// kSymCells cells on. Row blocks per workgroup: the most of 16, 8, 4 that
// still leaves at least 512 workgroups (measured best at 4,096, 8,192 and
// 16,384 cells; the column sums' lane reduction is paid once per workgroup's
// share). Simplified networks that sum_once picks get the group sums' room.
void build_sym(infoli_ctx* c) {
    int64_t total = 0;
    for (int k = 0; k < c->n_inst; ++k) {
        InstDesc& d = c->inst[k];
        d.sym = 0;
        d.psym_off = 0;
        d.sym_ki = 0;
        // by default only a lone network: in a batch the ordered tiles share one
        // launch with the other networks' tiles, which measured faster than the
        // pair kernel running ahead of that launch (Table 4's batches of 5,760
        // and 7,680 cells: 41.6 / 61.8 us per step against 47.5 / 70.5)
        if (d.sgj) {
            if (!sum_once(c, d)) continue;
            d.sym = 1;
            d.psym_off = total;
            total += vsum_floats(d.n);
            continue;
        }
        const bool want = c->opt.pair_path == 2 || (c->opt.pair_path == 0 && d.n >= kSymCells && c->n_inst == 1);
        if (d.conn != CONN_UNIFORM || !want || c->opt.step_mode == INFOLI_MODE_PERSISTENT) continue;
        d.sym = 1;
        d.psym_off = total;
        d.sym_ki = 4;
        for (int ki : {kSymMaxKi, kSymMaxKi / 2})
            if ((int64_t)sym_blocks(d.n) * sym_shares(d.n, ki) >= 512) {
                d.sym_ki = ki;
                break;
            }
        total += sym_floats(d.n, d.sym_ki);
    }
    if (total == 0) return;
    c->d_psym = c->alloc<float>((size_t)total);
    HIPX(hipMemset(c->d_psym, 0, sizeof(float) * (size_t)total));
    HIPX(hipMemcpy(c->d_inst, c->inst.data(), sizeof(InstDesc) * c->n_inst, hipMemcpyHostToDevice));
    HIPX(hipDeviceSynchronize());
}

void build_chunks(infoli_ctx* c, const infoli_network_spec* specs) {
    const int C = c->blk_cols;
    int64_t nca = 0, ncb = 0, nchunks = 0;
    bool any_w = false;
    auto chunks_of = [](int64_t cnt) { return (cnt + kChunkCols - 1) / kChunkCols; };
    for (int k = 0; k < c->n_inst; ++k) {
        InstDesc& d = c->inst[k];
        d.ca_off = d.cb_off = d.chk_off = d.chkb_off = -1;
        const infoli_network_spec& s = specs[k];
        if (d.conn != CONN_CSR || s.nnz == 0) continue;
        any_w = any_w || d.has_w;
        if (d.n <= 65536) {
            int64_t ch = 0;
            for (int i = 0; i < d.n; ++i) ch += chunks_of(s.row_ptr[i + 1] - s.row_ptr[i]);
            if (ch > INT32_MAX) continue;
            d.ca_off = nca;
            nca += d.n + 1;
            d.chk_off = nchunks;
            nchunks += ch;
        }
        if (d.blk_off >= 0 && C + kSelfSlots <= 65536) {
            int64_t ch = 0;
            for (int i = 0; i < d.n; ++i) {
                int64_t e = s.row_ptr[i];
                for (int b = 0; b < d.nblk; ++b) {
                    const int64_t e0 = e;
                    while (e < s.row_ptr[i + 1] && s.col[e] < (int64_t)(b + 1) * C) ++e;
                    ch += chunks_of(e - e0);
                }
            }
            if (ch > INT32_MAX) continue;
            d.cb_off = ncb;
            ncb += (int64_t)d.nblk * (d.n + 1);
            d.chkb_off = nchunks;
            nchunks += ch;
        }
    }
    if (nchunks == 0) return;
    std::vector<uint16_t> hc((size_t)nchunks * kChunkCols);
    std::vector<float> hw(any_w ? (size_t)nchunks * kChunkCols : 1, 0.0f);
    std::vector<int32_t> ha((size_t)std::max<int64_t>(nca, 1)), hb((size_t)std::max<int64_t>(ncb, 1));
    for (int k = 0; k < c->n_inst; ++k) {
        const InstDesc& d = c->inst[k];
        const infoli_network_spec& s = specs[k];
        if (d.ca_off >= 0) {
            int64_t pos = 0;   // chunk index relative to the network's first
            for (int i = 0; i < d.n; ++i) {
                ha[(size_t)(d.ca_off + i)] = (int32_t)pos;
                const int64_t rs = s.row_ptr[i], cnt = s.row_ptr[i + 1] - rs;
                const int64_t base = (d.chk_off + pos) * kChunkCols;
                for (int64_t e = 0; e < chunks_of(cnt) * kChunkCols; ++e) {
                    hc[(size_t)(base + e)] = (uint16_t)(e < cnt ? s.col[rs + e] : i);
                    if (d.has_w) hw[(size_t)(base + e)] = e < cnt ? s.w_csr[rs + e] : 0.0f;
                }
                pos += chunks_of(cnt);
            }
            ha[(size_t)(d.ca_off + d.n)] = (int32_t)pos;
        }
        if (d.cb_off >= 0) {
            // block-major: every row's segment of column block 0, then of
            // block 1, ...; a tile's pass over one block reads one contiguous
            // run, and no cache line is shared between two passes. Table
            // [nblk][n + 1]: the start of row i's segment in block b; row
            // i + 1's start ends it.
            std::vector<int64_t> bnd((size_t)d.n * (d.nblk + 1));   // per row, edge index at each block start
            for (int i = 0; i < d.n; ++i) {
                int64_t e = s.row_ptr[i];
                for (int b = 0; b < d.nblk; ++b) {
                    bnd[(size_t)i * (d.nblk + 1) + b] = e;
                    while (e < s.row_ptr[i + 1] && s.col[e] < (int64_t)(b + 1) * C) ++e;
                }
                bnd[(size_t)i * (d.nblk + 1) + d.nblk] = e;
            }
            int64_t pos = 0;
            for (int b = 0; b < d.nblk; ++b) {
                for (int i = 0; i < d.n; ++i) {
                    hb[(size_t)(d.cb_off + (int64_t)b * (d.n + 1) + i)] = (int32_t)pos;
                    const uint16_t pad = (uint16_t)(C + (i & (kSelfSlots - 1)));
                    const int64_t e0 = bnd[(size_t)i * (d.nblk + 1) + b];
                    const int64_t cnt = bnd[(size_t)i * (d.nblk + 1) + b + 1] - e0;
                    const int64_t base = (d.chkb_off + pos) * kChunkCols;
                    for (int64_t x = 0; x < chunks_of(cnt) * kChunkCols; ++x) {
                        hc[(size_t)(base + x)] = x < cnt ? (uint16_t)(s.col[e0 + x] - (int64_t)b * C) : pad;
                        if (d.has_w) hw[(size_t)(base + x)] = x < cnt ? s.w_csr[e0 + x] : 0.0f;
                    }
                    pos += chunks_of(cnt);
                }
                hb[(size_t)(d.cb_off + (int64_t)b * (d.n + 1) + d.n)] = (int32_t)pos;
            }
        }
    }
    // Bank-aware order of each chunk's eight columns (blocks layout, one
    // weight g): the chunk stream reads a tile's run in sweeps of 64
    // consecutive chunks from the run's start (tiles of kSelfSlots rows), lane
    // l the l-th chunk, and its e-th gather reads every lane's e-th column. A
    // chunk's columns may come in any order (only the order of the row's sum
    // changes), so each sweep's chunks are given orders under which each
    // gather's 64 slots fall on distinct LDS banks (slot mod 64), and each
    // half-wave's on distinct slot mod 32, as far as a greedy pass finds.
    for (int k = 0; k < c->n_inst; ++k) {
        const InstDesc& d = c->inst[k];
        if (d.cb_off < 0 || d.has_w) continue;
        for (int b = 0; b < d.nblk; ++b) {
            const int32_t* off = &hb[(size_t)(d.cb_off + (int64_t)b * (d.n + 1))];
            for (int r = 0; r < d.n; r += kSelfSlots) {
                const int64_t x0 = off[r], x1 = off[std::min(d.n, r + kSelfSlots)];
                for (int64_t w0 = x0; w0 < x1; w0 += 64) {
                    const int nch = (int)std::min<int64_t>(64, x1 - w0);
                    uint16_t* base = &hc[(size_t)(d.chkb_off + w0) * kChunkCols];
                    uint16_t out[64][kChunkCols];
                    bool used[64][kChunkCols] = {};
                    for (int e = 0; e < kChunkCols; ++e) {
                        int c64[64] = {}, c32[2][32] = {};
                        for (int l = 0; l < nch; ++l) {
                            int best = -1, cost = 1 << 30;
                            for (int u = 0; u < kChunkCols; ++u) {
                                if (used[l][u]) continue;
                                const int sl = base[l * kChunkCols + u];
                                const int cu = 4 * c64[sl & 63] + c32[l >> 5][sl & 31];
                                if (cu < cost) cost = cu, best = u;
                            }
                            used[l][best] = true;
                            const int sl = base[l * kChunkCols + best];
                            out[l][e] = (uint16_t)sl;
                            ++c64[sl & 63];
                            ++c32[l >> 5][sl & 31];
                        }
                    }
                    for (int l = 0; l < nch; ++l)
                        for (int e = 0; e < kChunkCols; ++e) base[l * kChunkCols + e] = out[l][e];
                }
            }
        }
    }
    // per chunk of the blocks layout, its row mod 256 (the chunk stream's row tag)
    std::vector<uint8_t> ht((size_t)nchunks, 0);
    for (int k = 0; k < c->n_inst; ++k) {
        const InstDesc& d = c->inst[k];
        if (d.cb_off < 0) continue;
        for (int b = 0; b < d.nblk; ++b)
            for (int i = 0; i < d.n; ++i)
                for (int32_t x = hb[(size_t)(d.cb_off + (int64_t)b * (d.n + 1) + i)];
                     x < hb[(size_t)(d.cb_off + (int64_t)b * (d.n + 1) + i + 1)]; ++x)
                    ht[(size_t)(d.chkb_off + x)] = (uint8_t)(i & (kSelfSlots - 1));
    }
    // the chunk stream loads whole items without clamping: both arrays carry
    // one item of zeroed slack after the last chunk
    const size_t slack = (size_t)kStreamSlack;
    c->d_rtag = c->alloc<uint8_t>((size_t)nchunks + slack);
    HIPX(hipMemcpy(c->d_rtag, ht.data(), ht.size(), hipMemcpyHostToDevice));
    HIPX(hipMemset(c->d_rtag + nchunks, 0, slack));
    c->d_chk = c->alloc<uint4>((size_t)nchunks + slack);
    HIPX(hipMemcpy(c->d_chk, hc.data(), sizeof(uint16_t) * hc.size(), hipMemcpyHostToDevice));
    HIPX(hipMemset(c->d_chk + nchunks, 0, sizeof(uint4) * slack));
    c->d_chkw = c->alloc<float>(hw.size());
    HIPX(hipMemcpy(c->d_chkw, hw.data(), sizeof(float) * hw.size(), hipMemcpyHostToDevice));
    c->d_ca = c->alloc<int32_t>(ha.size());
    HIPX(hipMemcpy(c->d_ca, ha.data(), sizeof(int32_t) * ha.size(), hipMemcpyHostToDevice));
    c->d_cb = c->alloc<int32_t>(hb.size());
    HIPX(hipMemcpy(c->d_cb, hb.data(), sizeof(int32_t) * hb.size(), hipMemcpyHostToDevice));
}

// ---------------------------------------------------------------- autotuner
// For every class of CSR network (log-spaced size and degree buckets) the
// candidate tile shapes (lanes per row, rows per tile, LDS staging of Vd) are
// timed on the network's own device data with dry launches (they write only
// the next-state buffer) replayed from graphs, as steps run, and the fastest
// is kept, in memory and in an
// on-disk cache (INFOLI_TUNE_CACHE, else ~/.cache/infoli-tune-v13.txt).
struct TuneChoice {
    int L, R, lds, bm;     // lanes per row, rows per tile, Vd in LDS,
                           // path (0 gathers, 1 bitmap, 2 blocked, 3 chunked gathers,
                           // 4 blocked chunk stream)
    int block;             // workgroup size timed (256 or 1024; the wide group may run 512)
    int rnd = kStreamRound;   // chunk stream: chunks per round (kStreamRound or half of it)
};

std::string tune_cache_path() {
    const char* p = std::getenv("INFOLI_TUNE_CACHE");
    if (p && *p) return p;
    const char* h = std::getenv("HOME");
    if (h && *h) return std::string(h) + "/.cache/infoli-tune-v14.txt";
    return "";
}

std::string tune_key(const infoli_ctx* c, const InstDesc& d, double deg) {
    const int nb = (int)std::ceil(std::log2((double)d.n) * 4.0);
    const int db = (int)std::ceil(std::log2(deg + 1.0) * 4.0);
    char buf[128];
    snprintf(buf, sizeof buf, "gfx950 groups2 c16=%d w=%d bits=%d blk=%d n%d d%d%s", d.col16, d.has_w,
             d.bits_off >= 0 ? 1 : 0, d.blk_off >= 0 ? c->blk_cols : 0, nb, db, d.sgj ? " sgj" : "");
    return buf;
}

// Whole-step launch modes: six bits (see the tuner below), so 0..63.
constexpr int kStepModes = 64;

// Lines "<class key>|L R lds bm block" (the class's best shape),
// "<class key>#256|..." (its best shape in 256-thread workgroups) and
// "ctx <hash>|mode" (the whole-step launch choice of one mix of networks).
std::map<std::string, TuneChoice> read_tune_cache(const std::string& path,
                                                  std::map<std::string, std::vector<int>>* modes) {
    std::map<std::string, TuneChoice> m;
    if (path.empty()) return m;
    std::FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return m;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char* bar = std::strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        if (std::strncmp(line, "ctx ", 4) == 0) {   // mode, then one refinement per class
            std::vector<int> v;
            char* p = bar + 1;
            char* end = nullptr;
            for (long x = std::strtol(p, &end, 10); end != p; x = std::strtol(p, &end, 10)) {
                v.push_back((int)x);
                p = end;
            }
            if (!v.empty() && v[0] >= 0 && v[0] < kStepModes) (*modes)[line] = v;
            continue;
        }
        TuneChoice t;
        if (std::sscanf(bar + 1, "%d %d %d %d %d %d", &t.L, &t.R, &t.lds, &t.bm, &t.block, &t.rnd) == 6 &&
            (t.block == 256 || t.block == 512 || t.block == 1024) && t.L >= 4 && t.L <= 1024 &&
            (t.rnd == kStreamRound || t.rnd == kStreamRound / 2) &&
            (t.L & (t.L - 1)) == 0 && t.R >= 1 && t.R <= kMaxTileRows && (t.lds == 0 || t.lds == 1) &&
            (t.bm >= 0 && t.bm <= 4))
            m[line] = t;
    }
    std::fclose(f);
    return m;
}

void append_tune_line(const std::string& path, const std::string& line) {
    if (path.empty()) return;
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) mkdir(path.substr(0, slash).c_str(), 0755);
    std::FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s\n", line.c_str());
    std::fclose(f);
}

// Optional record of the tuner's timings (INFOLI_TUNE_LOG: a file the
// lines are appended to), for checking what a run chose and why.
void tune_log(const char* fmt, ...) {
    const char* p = std::getenv("INFOLI_TUNE_LOG");
    if (!p || !*p) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    append_tune_line(p, buf);
}

void append_tune_cache(const std::string& path, const std::string& key, const TuneChoice& t) {
    char buf[64];
    snprintf(buf, sizeof buf, "|%d %d %d %d %d %d", t.L, t.R, t.lds, t.bm, t.block, t.rnd);
    append_tune_line(path, key + buf);
}

// Device time of one repetition of `launch` (which queues one step's dry
// launches on the stream it is given, reading the state buffer of the parity
// it is given) as the library runs steps: `reps` (even) repetitions captured
// into a graph, alternating the state buffers as consecutive steps do (each
// reads what the previous one wrote), the graph replayed `trials` times after
// one warm-up replay, the fastest replay kept. Host-launched repetitions of a
// step of a few microseconds measure the host's launch rate as much as the
// kernels and ranked shapes differently from box to box; repetitions that all
// read one buffer timed about 2 us under the real step of the 4,096-cell mix.
template <typename F>
float time_replayed(infoli_ctx* c, F&& launch, int reps, int trials) {
    hipGraph_t g = nullptr;
    HIPX(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int w = 0; w < reps; ++w) launch(c->cap_stream, c->cur ^ (w & 1));
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess) fail(INFOLI_E_DEVICE, "tuning capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) fail(INFOLI_E_DEVICE, "tuning graph instantiation failed: %s", hipGetErrorString(e));
    struct Release {       // on every exit: the replays drained, then the graph destroyed
        infoli_ctx* c;
        hipGraphExec_t ex;
        ~Release() {
            (void)hipStreamSynchronize(c->stream);
            (void)hipGraphExecDestroy(ex);
        }
    } release{c, ex};
    HIPX(hipGraphLaunch(ex, c->stream));
    float best = 1e30f;
    for (int t = 0; t < trials; ++t) {
        HIPX(hipEventRecord(c->ev0, c->stream));
        HIPX(hipGraphLaunch(ex, c->stream));
        HIPX(hipEventRecord(c->ev1, c->stream));
        HIPX(hipEventSynchronize(c->ev1));
        float ms = 0.0f;
        HIPX(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        best = std::min(best, ms / reps);
    }
    return best;
}

// Duration of a dry launch of the tiles of networks `ks` (one size and
// degree class) shaped by t, replayed from a graph.
float time_shape(infoli_ctx* c, const std::vector<int>& ks, const TuneChoice& t, Tile* d_tmp) {
    std::vector<std::pair<double, Tile>> planned;
    size_t lds = 16;
    int var = t.bm == 4 ? kVarStream : kVarNoW;   // the variant the step will launch these tiles with
    for (int k : ks) {
        InstDesc d = c->inst[k];
        if (d.has_w || d.pcell) var = kVarAll;
        d.lanes_per_row = t.L;
        d.vd_lds = t.lds;
        d.bitmap = t.bm == 1;
        d.blocked = t.bm == 2 || t.bm == 4;
        d.stream = t.bm == 4;
        d.stream_round = t.bm == 4 ? t.rnd : kStreamRound;
        d.chunked = t.bm == 3;
        HIPX(hipMemcpy(c->d_inst + k, &d, sizeof(d), hipMemcpyHostToDevice));
        append_tiles(planned, k, d.n, t.R, 0.0);
        if (t.bm == 1) lds = std::max(lds, ((bitmap_lds_floats(d.n) + 3) / 4) * sizeof(float4));
        else if (t.bm == 2)
            lds = std::max(lds, ((size_t)(c->blk_cols + kSelfSlots + 3) / 4) * sizeof(float4));
        else if (t.bm == 4)
            lds = std::max(lds, ((lds_floats_for(c, d, t.block) + 3) / 4) * sizeof(float4));
        else if (t.lds) lds = std::max(lds, ((size_t)(d.n + 3) / 4) * sizeof(float4));
    }
    std::vector<Tile> tl;
    for (const auto& pt : planned) tl.push_back(pt.second);
    HIPX(hipMemcpy(d_tmp, tl.data(), sizeof(Tile) * tl.size(), hipMemcpyHostToDevice));
    StepArgs a = make_args(c, false);
    a.tiles = d_tmp;
    a.dry = 1;
    const int block = t.block;
    const unsigned ntiles = (unsigned)tl.size();
    return time_replayed(
        c, [&](hipStream_t st, int from) { launch_tiles(c, st, a, block, ntiles, lds, from, c->step, 0, var); }, 10,
        3);
}

// Timings within kTieMargin of the fastest count as equal; among those the
// choice follows a fixed preference, so that runs on different boxes (and
// timing noise) agree.
constexpr float kTieMargin = 0.03f;

// Preference among equally fast shapes: chunk stream, bitmap, chunked
// gathers, gathers, column blocks; then the wider workgroup; then fewer
// lanes per row, fewer rows, no LDS staging; then the smaller round of the
// chunk stream (its rounds of 4,096 chunks timed 3-4 % faster than 8,192 at
// 65,536 cells of degree 1,000, close to the margin).
int64_t pref_key(const TuneChoice& t) {
    static const int rank[5] = {3, 1, 4, 2, 0};   // by bm: 0 gathers .. 4 stream
    return (((((int64_t)rank[t.bm] * 2 + (t.block == 256 ? 1 : 0)) * 1024 + t.L) * 1024 + t.R) * 2 + t.lds) * 2 +
           (t.rnd < kStreamRound ? 0 : 1);
}

// The preferred entry among those within kTieMargin of the fastest; none
// (block 0) when v is empty.
TuneChoice pick_shape(const std::vector<std::pair<float, TuneChoice>>& v) {
    TuneChoice none{0, 0, 0, 0, 0};
    if (v.empty()) return none;
    float best = 1e30f;
    for (const auto& e : v) best = std::min(best, e.first);
    const TuneChoice* pick = nullptr;
    for (const auto& e : v)
        if (e.first <= best * (1.0f + kTieMargin) && (!pick || pref_key(e.second) < pref_key(*pick)))
            pick = &e.second;
    return *pick;
}

void apply_choice(infoli_ctx* c, const std::vector<int>& ks, TuneChoice best) {
    for (int k : ks)   // a cached choice this context cannot honour falls back to gathers
        if ((best.bm == 1 && c->inst[k].bits_off < 0) || (best.bm == 2 && c->inst[k].blk_off < 0) ||
            (best.bm == 3 && c->inst[k].ca_off < 0) || (best.bm == 4 && c->inst[k].cb_off < 0))
            best = TuneChoice{std::min(best.L, 256), std::max(1, 256 / std::min(best.L, 256)), 0, 0, 256};
    for (int k : ks) {
        c->inst[k].lanes_per_row = best.L;
        c->inst[k].vd_lds = best.lds;
        c->inst[k].bitmap = best.bm == 1;
        c->inst[k].blocked = best.bm == 2 || best.bm == 4;
        c->inst[k].stream = best.bm == 4;
        c->inst[k].stream_round = best.bm == 4 ? best.rnd : kStreamRound;
        c->inst[k].chunked = best.bm == 3;
        c->inst[k].wide = best.block == 1024;
        c->rows_of[k] = best.R;
    }
}

// Duration of a dry whole step (both launch groups) as finalised, replayed
// from a graph: the fastest of four replays of 20 steps.
float time_step(infoli_ctx* c, bool fork) {
    StepArgs a = make_args(c, false);
    a.dry = 1;
    return time_replayed(c, [&](hipStream_t st, int from) { launch_groups(c, st, a, from, c->step, 0, fork); }, 20,
                         4);
}

uint64_t fnv1a(const std::string& s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    return h;
}

// Per size/degree class of CSR network, the tile shape and path with the
// shortest dry launch of that class alone (its best overall and its best in
// 256-thread workgroups); then, for the whole mix of networks, the faster of
// the per-class best shapes and the all-256 shapes, with the two launch
// groups as concurrent branches or one after the other, timed as whole steps.
void autotune_shapes(infoli_ctx* c) {
    if (c->opt.lanes_per_row || c->opt.tile_rows) return;   // shapes given by the caller
    const std::string path = tune_cache_path();
    std::map<std::string, TuneChoice> cache;
    std::map<std::string, std::vector<int>> modes;
    if (c->opt.autotune == 1) cache = read_tune_cache(path, &modes);
    // classes of CSR networks
    std::map<std::string, std::vector<int>> classes;
    for (int k = 0; k < c->n_inst; ++k) {
        const InstDesc& d = c->inst[k];
        if (d.conn != CONN_CSR || c->deg_of[k] <= 0.0) continue;
        classes[tune_key(c, d, c->deg_of[k])].push_back(k);
    }
    Tile* d_tmp = nullptr;
    constexpr int kAlts = 8;
    struct ClassChoice {
        TuneChoice best, best256, best256nc;   // overall; in 256 threads; in 256 threads, not chunked
        TuneChoice best1024;                   // in 1024 threads (block 0: none timed)
        TuneChoice bm256, bm1024;              // the bitmap path in 256 / 1024 threads (block 0: none)
        TuneChoice alt[kAlts];                 // the fastest distinct 256-thread shapes, fastest first
        int nalt = 0;
    };
    std::map<std::string, ClassChoice> chosen;
    for (const auto& kv : classes) {
        const std::string& key = kv.first;
        const std::vector<int>& ks = kv.second;
        TuneChoice best{0, 0, 0, 0, 256}, best256{0, 0, 0, 0, 256}, best256nc{0, 0, 0, 0, 256};
        TuneChoice best1024{0, 0, 0, 0, 0};
        TuneChoice bm256{0, 0, 0, 0, 0}, bm1024{0, 0, 0, 0, 0};
        ClassChoice cc;
        auto hit = cache.find(key);
        auto hit256 = cache.find(key + "#256");
        auto hitnc = cache.find(key + "#256nc");
        auto hita = cache.find(key + "#a0");
        auto hit1024 = cache.find(key + "#1024");
        if (hit != cache.end() && hit256 != cache.end() && hitnc != cache.end() && hita != cache.end() &&
            hit1024 != cache.end() && hit1024->second.L <= 256 &&
            hit->second.L <= 256 && hit256->second.L <= 256 && hit256->second.block == 256 &&
            hitnc->second.L <= 256 && hitnc->second.block == 256 && hitnc->second.bm != 3) {
            best = hit->second;
            best256 = hit256->second;
            best256nc = hitnc->second;
            best1024 = hit1024->second;
            auto hb = cache.find(key + "#bm256");
            if (hb != cache.end() && hb->second.bm == 1 && hb->second.block == 256) bm256 = hb->second;
            hb = cache.find(key + "#bm1024");
            if (hb != cache.end() && hb->second.bm == 1 && hb->second.block == 1024) bm1024 = hb->second;
            for (int a = 0; a < kAlts; ++a) {
                auto h = cache.find(key + "#a" + std::to_string(a));
                if (h == cache.end() || h->second.block != 256 || h->second.L > 256) break;
                cc.alt[cc.nalt++] = h->second;
            }
            c->tune_cached += (int)ks.size();
        } else {
            if (!d_tmp) d_tmp = c->alloc<Tile>(c->total_cells + 1);
            // representative size and degree of the class
            int n = 0;
            double deg = 0.0;
            for (int k : ks) {
                n = std::max(n, c->inst[k].n);
                deg = std::max(deg, c->deg_of[k]);
            }
            std::vector<std::pair<float, TuneChoice>> timed, all, all256, all256nc, all1024;
            bool all_rows = c->d_ca != nullptr;    // every network of the class has the chunked rows layout
            for (int k : ks) all_rows = all_rows && c->inst[k].ca_off >= 0;
            // every shape timed; the class's choices picked at the end (ties
            // by the fixed preference), best256 also as the search goes on
            auto consider = [&](const TuneChoice& t) {
                const float ms = time_shape(c, ks, t, d_tmp);
                tune_log("class %s shape L%d R%d lds%d path%d block%d round%d: %.2f us", key.c_str(), t.L, t.R, t.lds,
                         t.bm, t.block, t.rnd, 1e3f * ms);
                all.push_back({ms, t});
                if (t.block == 256) {
                    timed.push_back({ms, t});
                    all256.push_back({ms, t});
                    if (t.bm != 3) all256nc.push_back({ms, t});
                    best256 = pick_shape(all256);
                }
                if (t.block == 1024) all1024.push_back({ms, t});
                if (t.bm == 1) (t.block == 256 ? bm256 : bm1024) = t;
            };
            for (int L = 4; L <= 256; L *= 2) {
                if (L > 4 && L > 2.0 * deg) break;
                if (deg / L > 256.0) continue;
                for (int m = 1; m <= 4; m *= 2) {
                    const int R = std::max(1, 256 / L) * m;
                    if (R > kMaxTileRows) continue;
                    for (int lds = 0; lds <= (n <= kChunk ? 1 : 0); ++lds) {
                        consider(TuneChoice{L, R, lds, 0, 256});
                        if (all_rows) consider(TuneChoice{L, R, lds, 3, 256});
                    }
                }
            }
            // the gathers in 1024-thread workgroups (at the best 256-thread
            // lane count and twice it), so that a step whose other networks
            // want 1024 threads can run as one launch
            for (int L : {best256.L, 2 * best256.L}) {
                if (L > 256 || (L > 4 && L > 2.0 * deg)) continue;
                for (int m = 1; m <= 2; m *= 2) {
                    const int R = std::max(1, 1024 / L) * m;
                    if (R > kMaxTileRows) continue;
                    consider(TuneChoice{L, R, best256.lds, 0, 1024});
                    if (all_rows) consider(TuneChoice{L, R, best256.lds, 3, 1024});
                }
            }
            // the bitmap path, when every network of the class has one
            bool all_bits = c->d_bits != nullptr;
            for (int k : ks) all_bits = all_bits && c->inst[k].bits_off >= 0;
            if (all_bits)
                for (int blk : {256, 1024}) consider(TuneChoice{best256.L, kBitRows, 0, 1, blk});
            // the blocked chunk stream, when every network of the class has the
            // chunked blocks layout and the device gives a workgroup its LDS
            bool all_cb = c->d_rtag != nullptr;
            for (int k : ks)
                all_cb = all_cb && c->inst[k].cb_off >= 0 && !c->inst[k].has_w && !c->inst[k].pcell &&
                         c->inst[k].nblk <= kStreamMaxBlocks && c->inst[k].cell_off % 4 == 0 && stream_ok(c);
            if (all_cb)
                for (int blk : {1024, 512}) {
                    InstDesc d = c->inst[ks[0]];
                    d.blocked = d.stream = 1;
                    if (lds_floats_for(c, d, blk) * sizeof(float) + kStaticLds <= (size_t)c->lds_max)
                        for (int rnd : {kStreamRound, kStreamRound / 2})
                            consider(TuneChoice{64, kSelfSlots, 0, 4, blk, rnd});
                }
            // the column-blocked path, when every network of the class has it
            bool all_blk = c->d_blk != nullptr;
            for (int k : ks) all_blk = all_blk && c->inst[k].blk_off >= 0;
            if (all_blk)
                for (int L = 8; L <= 64; L *= 2) {
                    if (L > 8 && L > 2.0 * deg / c->inst[ks[0]].nblk) break;
                    for (int m = 1; m <= kBlkPasses; m *= 2) {
                        const int R = (1024 / L) * m;
                        if (R > kMaxTileRows) continue;
                        consider(TuneChoice{L, R, 0, 2, 1024});
                    }
                }
            best = pick_shape(all);
            if (!all256.empty()) best256 = pick_shape(all256);
            if (!all256nc.empty()) best256nc = pick_shape(all256nc);
            if (!all1024.empty()) best1024 = pick_shape(all1024);
            std::stable_sort(timed.begin(), timed.end(),
                             [](const auto& x, const auto& y) { return x.first < y.first; });
            for (const auto& tt : timed) {
                if (cc.nalt == kAlts) break;
                cc.alt[cc.nalt++] = tt.second;
            }
            append_tune_cache(path, key, best);
            append_tune_cache(path, key + "#256", best256);
            append_tune_cache(path, key + "#256nc", best256nc);
            append_tune_cache(path, key + "#1024", best1024);
            if (bm256.block) append_tune_cache(path, key + "#bm256", bm256);
            if (bm1024.block) append_tune_cache(path, key + "#bm1024", bm1024);
            for (int a = 0; a < cc.nalt; ++a) append_tune_cache(path, key + "#a" + std::to_string(a), cc.alt[a]);
            c->tuned += (int)ks.size();
        }
        cc.best = best;
        cc.best256 = best256;
        cc.best256nc = best256nc;
        cc.best1024 = best1024;
        cc.bm256 = bm256;
        cc.bm1024 = bm1024;
        chosen[key] = cc;
    }

    // whole-step choice for this mix of networks
    std::vector<std::string> parts;
    for (int k = 0; k < c->n_inst; ++k) {
        const InstDesc& d = c->inst[k];
        char buf[64];
        snprintf(buf, sizeof buf, "%d:%d:%d", d.conn, d.n, group_for(d));
        parts.push_back(d.conn == CONN_CSR && c->deg_of[k] > 0.0 ? tune_key(c, d, c->deg_of[k]) : buf);
    }
    std::sort(parts.begin(), parts.end());
    std::string sig;
    for (const auto& p : parts) sig += p + ";";
    char ctx_key[64];
    snprintf(ctx_key, sizeof ctx_key, "ctx %016llx", (unsigned long long)fnv1a(sig));
    // variant of the per-class choices: bit 0, each class in its best
    // 256-thread shape; bit 3, each class in its best 1024-thread shape;
    // bit 2, chunked gathers in 256 threads replaced by the best
    // non-chunked 256-thread shape; bit 5, every class that has a bitmap
    // shape takes it (in 1024 threads under bit 3 when timed, else in 256):
    // timed alone a class can rank the bitmap and its gathers differently
    // from the whole step
    auto pick = [&](const ClassChoice& ch, int m) {
        if ((m & 32) && (ch.bm256.block || ch.bm1024.block))
            return ((m & 8) && ch.bm1024.block) || !ch.bm256.block ? ch.bm1024 : ch.bm256;
        TuneChoice t = (m & 8) && ch.best1024.block == 1024 ? ch.best1024 : (m & 1) ? ch.best256 : ch.best;
        if ((m & 4) && t.bm == 3 && t.block == 256) t = ch.best256nc;
        return t;
    };
    // the wide group's workgroup size under mode m (an explicit option wins)
    auto wide_block = [&](int m) { return c->opt.wide_threads ? c->opt.wide_threads : (m & 16) ? 512 : 1024; };
    auto apply_all = [&](int m) {
        for (const auto& kv : classes) apply_choice(c, kv.second, pick(chosen[kv.first], m));
        // bit 3 also moves every all-to-all network into the wide group
        for (int k = 0; k < c->n_inst; ++k)
            if (c->inst[k].conn == CONN_UNIFORM) c->inst[k].wide = (m & 8) ? 1 : 0;
    };
    // bits 0, 2, 3 and 5 as above; bit 1: the two launch groups one after the
    // other; bit 4: the wide launch group in 512-thread workgroups (two per
    // compute unit, so one can stage a column block while the other gathers)
    int mode = 0;
    const int ncls = (int)classes.size();
    std::vector<int> refine(ncls, -1);   // per class: -1 its mode choice, else that alternative
    auto mh = modes.find(ctx_key);
    if (mh != modes.end() && (int)mh->second.size() == 1 + ncls) {
        mode = mh->second[0];
        for (int i = 0; i < ncls; ++i) refine[i] = mh->second[1 + i];
    } else {
        bool wide = false, chunk = false, narrow = false, bits = false;   // variants that change something
        for (const auto& kv : chosen) {
            bits = bits || kv.second.bm256.block || kv.second.bm1024.block;
            wide = wide || kv.second.best.block != 256;
            narrow = narrow || (kv.second.best.block == 256 && kv.second.best1024.block == 1024);
            chunk = chunk || kv.second.best.bm == 3 || kv.second.best256.bm == 3;
        }
        // every variant timed in two interleaved rounds, the smaller kept
        float mode_ms[kStepModes];
        for (float& v : mode_ms) v = 1e30f;
        for (int round = 0; round < 2; ++round)
            for (int m = 0; m < kStepModes; ++m) {
                if (((m & 1) && !wide) || ((m & 4) && !chunk) || ((m & 8) && (!narrow || (m & 1)))) continue;
                if ((m & 32) && !bits) continue;
                if ((m & 16) && c->opt.wide_threads) continue;
                apply_all(m);
                c->grp[1].block = wide_block(m);
                finalize_tiles(c);
                const bool both = !c->grp[0].tiles.empty() && !c->grp[1].tiles.empty();
                if ((m & 2) && !both) continue;
                if ((m & 16) && c->grp[1].tiles.empty()) continue;
                mode_ms[m] = std::min(mode_ms[m], time_step(c, !(m & 2)));
                tune_log("step mode %d round %d: %.2f us", m, round, 1e3f * mode_ms[m]);
            }
        // the modes within 10 % of the fastest timed again, interleaved,
        // three more rounds; then within kTieMargin the lowest mode number
        // (the plainer arrangement) wins
        float fastest = 1e30f;
        for (int m = 0; m < kStepModes; ++m) fastest = std::min(fastest, mode_ms[m]);
        std::vector<int> close;
        for (int m = 0; m < kStepModes; ++m)
            if (mode_ms[m] <= 1.10f * fastest) close.push_back(m);
        if (close.size() > 1)
            for (int round = 0; round < 3; ++round)
                for (int m : close) {
                    apply_all(m);
                    c->grp[1].block = wide_block(m);
                    finalize_tiles(c);
                    mode_ms[m] = std::min(mode_ms[m], time_step(c, !(m & 2)));
                    tune_log("step mode %d retimed: %.2f us", m, 1e3f * mode_ms[m]);
                }
        fastest = 1e30f;
        for (int m : close) fastest = std::min(fastest, mode_ms[m]);
        mode = close.empty() ? 0 : close.back();
        for (int m : close)
            if (mode_ms[m] <= fastest * (1.0f + kTieMargin)) {
                mode = m;
                break;
            }
        // Refinement in the whole step: a class timed alone can rank shapes
        // differently from the full step. Every class with at least 5 % of
        // the step's pairs tries its fastest 256-thread alternatives with
        // the others fixed; a change stays when the step is 2 % faster.
        apply_all(mode);
        c->grp[1].block = wide_block(mode);
        finalize_tiles(c);
        double total = 0.0;
        std::vector<std::pair<double, int>> order;
        int i = 0;
        for (const auto& kv : classes) {
            double pairs = 0.0;
            for (int k : kv.second) pairs += c->deg_of[k] * c->inst[k].n;
            order.push_back({pairs, i++});
            total += pairs;
        }
        std::sort(order.begin(), order.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
        std::vector<std::string> keys;
        for (const auto& kv : classes) keys.push_back(kv.first);
        for (const auto& o : order) {
            if (o.first < 0.05 * total) break;
            const std::string& key = keys[o.second];
            const ClassChoice& ch = chosen[key];
            const TuneChoice base = pick(ch, mode);
            for (int a = 0; a < ch.nalt; ++a) {
                const TuneChoice& t = ch.alt[a];
                const TuneChoice& now = refine[o.second] >= 0 ? ch.alt[refine[o.second]] : base;
                if (t.L == now.L && t.R == now.R && t.lds == now.lds && t.bm == now.bm && t.block == now.block)
                    continue;
                // the current choice and the alternative, timed back to back twice
                float cur_ms = 1e30f, alt_ms = 1e30f;
                for (int round = 0; round < 2; ++round) {
                    apply_choice(c, classes[key], now);
                    finalize_tiles(c);
                    cur_ms = std::min(cur_ms, time_step(c, !(mode & 2)));
                    apply_choice(c, classes[key], t);
                    finalize_tiles(c);
                    alt_ms = std::min(alt_ms, time_step(c, !(mode & 2)));
                }
                if (alt_ms < (1.0f - kTieMargin) * cur_ms) refine[o.second] = a;
                else apply_choice(c, classes[key], now);
            }
        }
        tune_log("step mode chosen: %d", mode);
        std::string line = ctx_key;
        line += "|" + std::to_string(mode);
        for (int r : refine) line += " " + std::to_string(r);
        append_tune_line(path, line);
    }
    apply_all(mode);
    c->grp[1].block = wide_block(mode);
    {
        int i = 0;
        for (const auto& kv : classes) {
            const int r = refine[i++];
            if (r >= 0 && r < chosen[kv.first].nalt) apply_choice(c, kv.second, chosen[kv.first].alt[r]);
        }
    }
    c->fork_groups = !(mode & 2);
    c->tune_mode = mode;
}

// The tuner's timed steps advance the state like real ones (they alternate
// the two buffers); the initial state is kept aside and put back afterwards.
void autotune(infoli_ctx* c) {
    const size_t bytes = sizeof(float) * NSV * (size_t)c->stride;
    struct Saved {         // on every exit: the stream drained, then the copy freed
        infoli_ctx* c;
        void* p = nullptr;
        ~Saved() {
            (void)hipStreamSynchronize(c->stream);
            if (p) (void)hipFree(p);
        }
    } sv{c};
    HIPX(hipMalloc(&sv.p, bytes));
    void* saved = sv.p;
    HIPX(hipMemcpyAsync(saved, c->state[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream));
    autotune_shapes(c);
    HIPX(hipMemcpyAsync(c->state[c->cur], saved, bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPX(hipStreamSynchronize(c->stream));
}

void launch_persistent(infoli_ctx* c, int64_t n_steps, bool dry = false);

// Dry timing of one persistent launch of kTimedSteps steps against as many
// tiled step launches (launch mode: an upper bound of a graph replay); true
// when the persistent kernel is faster. State buffers are rewritten by the
// first real step, nothing else is touched.
bool time_persistent_vs_tiles(infoli_ctx* c) {
    constexpr int kTimedSteps = 40;
    StepArgs a = make_args(c, false);
    a.dry = 1;
    float best_p = 1e30f, best_t = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        HIPX(hipEventRecord(c->ev0, c->stream));
        launch_persistent(c, kTimedSteps, true);
        HIPX(hipEventRecord(c->ev1, c->stream));
        HIPX(hipEventSynchronize(c->ev1));
        float ms = 0.0f;
        HIPX(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        best_p = std::min(best_p, ms);
        HIPX(hipEventRecord(c->ev0, c->stream));
        for (int k = 0; k < kTimedSteps; ++k) launch_groups(c, c->stream, a, c->cur, c->step, 0, false);
        HIPX(hipEventRecord(c->ev1, c->stream));
        HIPX(hipEventSynchronize(c->ev1));
        HIPX(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        best_t = std::min(best_t, ms);
    }
    HIPX(hipGetLastError());
    return best_p <= best_t;
}

void build_context(infoli_ctx* c, const infoli_network_spec* specs, int32_t ninst,
                   const infoli_options* opt) {
    if (!specs || ninst < 1) fail(INFOLI_E_INVALID_ARG, "need at least one network spec");
    infoli_default_options(&c->opt);
    if (opt) c->opt = *opt;
    if (c->opt.step_mode < 0 || c->opt.step_mode > INFOLI_MODE_PERSISTENT)
        fail(INFOLI_E_INVALID_ARG, "unknown step_mode %d", c->opt.step_mode);
    if (c->opt.graph_chunk < 2 || (c->opt.graph_chunk & 1))
        fail(INFOLI_E_INVALID_ARG, "graph_chunk must be even and >= 2");
    if (c->opt.max_spikes_per_cell < 0 || c->opt.max_spikes_per_cell > 4096)
        fail(INFOLI_E_INVALID_ARG, "max_spikes_per_cell must be in [0, 4096]");
    if (c->opt.lanes_per_row != 0 &&
        (c->opt.lanes_per_row < 4 || c->opt.lanes_per_row > 256 ||
         (c->opt.lanes_per_row & (c->opt.lanes_per_row - 1))))
        fail(INFOLI_E_INVALID_ARG, "lanes_per_row must be 0 or a power of two in [4, 256]");
    if (c->opt.autotune < 0 || c->opt.autotune > 2)
        fail(INFOLI_E_INVALID_ARG, "autotune must be 0, 1 or 2");
    if (c->opt.csr_path < 0 || c->opt.csr_path > 5)
        fail(INFOLI_E_INVALID_ARG, "csr_path must be 0, 1, 2, 3, 4 or 5");
    if (c->opt.tile_rows < 0 || c->opt.tile_rows > kMaxTileRows)
        fail(INFOLI_E_INVALID_ARG, "tile_rows must be in [0, %d]", kMaxTileRows);
    if (c->opt.output_ring_steps < 0 || c->opt.output_ring_steps > (1 << 20))
        fail(INFOLI_E_INVALID_ARG, "output_ring_steps must be in [0, 2^20]");
    if (c->opt.wide_threads != 0 && c->opt.wide_threads != 512 && c->opt.wide_threads != 1024)
        fail(INFOLI_E_INVALID_ARG, "wide_threads must be 0, 512 or 1024");
    if (c->opt.pair_path < 0 || c->opt.pair_path > 2) fail(INFOLI_E_INVALID_ARG, "pair_path must be 0, 1 or 2");
    for (int k = 0; k < ninst; ++k) validate_spec(specs[k], k);
    for (int k = 1; k < ninst; ++k) {
        if (specs[k].step0 != specs[0].step0) fail(INFOLI_E_INVALID_ARG, "all networks must share step0");
        if (specs[k].dt_ms != specs[0].dt_ms) fail(INFOLI_E_INVALID_ARG, "all networks must share dt_ms");
    }

    int dev = 0;
    HIPX(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPX(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        fail(INFOLI_E_DEVICE, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);

    c->n_inst = ninst;
    c->n_cu = std::max(1, prop.multiProcessorCount);
    c->dt = specs[0].dt_ms;
    c->step = specs[0].step0;
    c->grp[0].block = 256;
    c->grp[1].block = c->opt.wide_threads ? c->opt.wide_threads : 1024;
    {
        int lds_max = 0;
        HIPX(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        // 16,384-cell blocks (64 KB) when the 1024-thread kernel's static LDS fits beside them
        c->blk_cols = lds_max >= 16384 * 4 + 8192 ? 16384 : 8192;
        c->lds_max = lds_max;
    }

    // ---- layout of the flattened networks
    int64_t cells = 0, rp_total = 0, w_total = 0, col_total = 0, stream_total = 0;
    int32_t pulses_total = 0;
    c->inst.resize(ninst);
    for (int k = 0; k < ninst; ++k) {
        const infoli_network_spec& s = specs[k];
        InstDesc& d = c->inst[k];
        std::memset(&d, 0, sizeof(d));
        d.cell_off = cells;
        d.n = s.n_cells;
        d.conn = s.conn;
        d.g = s.g_uniform;
        d.sgj = s.gap_kind == INFOLI_GAP_SIMPLIFIED ? 1 : 0;
        d.pcell = s.cell_params ? 1 : 0;
        d.stream_off = -1;
        d.stream_round = kStreamRound;
        std::memcpy(&d.p, s.params ? s.params : kDefaultParams, sizeof(CellParams));
        cells += s.n_cells;
        if (s.conn == INFOLI_CONN_DENSE) {
            d.w_off = w_total;
            w_total += (int64_t)s.n_cells * s.n_cells;
            c->pairs_per_step += (int64_t)s.n_cells * s.n_cells;
        } else if (s.conn == INFOLI_CONN_CSR) {
            d.rp_off = rp_total;
            rp_total += s.n_cells + 1;
            d.w_off = col_total;
            col_total += s.nnz;
            d.has_w = s.w_csr ? 1 : 0;
            const double deg = (double)s.nnz / s.n_cells;
            d.lanes_per_row = std::min(256, c->opt.lanes_per_row ? c->opt.lanes_per_row : pick_lanes(deg, 256));
            c->pairs_per_step += s.nnz;
        } else if (s.conn == INFOLI_CONN_UNIFORM_ALL) {
            c->pairs_per_step += (int64_t)s.n_cells * (s.n_cells - 1);
        }
        d.pulse_off = pulses_total;
        d.n_pulses = s.n_pulses;
        pulses_total += s.n_pulses;
        if (s.i_stream) {
            d.stream_off = stream_total;
            d.stream_steps = s.i_stream_steps;
            stream_total += s.i_stream_steps * s.n_cells;
        }
    }
    if (w_total > 0 && col_total > 0)
        fail(INFOLI_E_UNSUPPORTED, "a batch may not mix DENSE and CSR networks");
    int32_t max_n = 0;
    for (int k = 0; k < ninst; ++k) max_n = std::max(max_n, specs[k].n_cells);
    if (c->opt.step_mode == INFOLI_MODE_PERSISTENT && max_n > kPersistCells)
        fail(INFOLI_E_UNSUPPORTED, "PERSISTENT mode holds networks of at most %d cells (largest: %d)",
             kPersistCells, max_n);
    bool cparams = false;
    for (int k = 0; k < ninst; ++k) cparams = cparams || specs[k].cell_params;
    if (c->opt.step_mode == INFOLI_MODE_PERSISTENT && cparams)
        fail(INFOLI_E_UNSUPPORTED, "PERSISTENT mode takes per-network parameters only");
    // AUTO with one real-time sized network: one persistent workgroup or the
    // tiled launches, whichever steps faster (timed below when autotuning,
    // else persistent only where a row is cheap for one thread to walk)
    bool persist_candidate = false;
    if (c->opt.step_mode == INFOLI_MODE_AUTO && ninst == 1 && max_n <= 1024 && !cparams) {
        const infoli_network_spec& s0 = specs[0];
        const bool cheap_rows = s0.conn == INFOLI_CONN_NONE || s0.conn == INFOLI_CONN_UNIFORM_ALL ||
                                (s0.conn == INFOLI_CONN_CSR && s0.nnz <= 8 * (int64_t)s0.n_cells);
        if (c->opt.autotune) persist_candidate = true;
        else if (cheap_rows) c->opt.step_mode = INFOLI_MODE_PERSISTENT;
    }
    c->persist_cpt = 1;
    while (c->persist_cpt * kPersistBlock < max_n) c->persist_cpt *= 2;
    c->total_cells = cells;
    c->stride = (cells + 63) & ~int64_t(63);

    // ---- per-network kernel layout and tiles (blocks of consecutive rows)
    bool col16 = col_total > 0;
    for (int k = 0; k < ninst; ++k)
        if (c->inst[k].conn == CONN_CSR && c->inst[k].n > 65536) col16 = false;
    c->rows_of.assign(ninst, kMaxTileRows);
    c->deg_of.assign(ninst, 0.0);
    for (int k = 0; k < ninst; ++k) {
        InstDesc& d = c->inst[k];
        int rows;
        switch (d.conn) {
            case CONN_UNIFORM:   // one row per lane; a row per thread when the sum is taken once
                rows = sum_once(c, d) ? kMaxTileRows : kUniformRows;
                c->deg_of[k] = d.n;
                break;
            case CONN_DENSE: rows = c->opt.tile_rows ? c->opt.tile_rows : 16; c->deg_of[k] = d.n; break;
            case CONN_CSR: {
                const double deg = (double)specs[k].nnz / d.n;
                c->deg_of[k] = deg;
                // one pass of row groups per tile: short dependent-load chains
                const int per_pass = std::max(1, 256 / d.lanes_per_row);
                rows = c->opt.tile_rows ? c->opt.tile_rows : std::min(kMaxTileRows, per_pass);
                d.col16 = col16 ? 1 : 0;
                d.vd_lds = (d.n <= kChunk && (double)rows * deg >= 2.0 * d.n) ? 1 : 0;
                break;
            }
            default: rows = c->opt.tile_rows ? c->opt.tile_rows : kMaxTileRows; break;
        }
        c->rows_of[k] = std::min(rows, kMaxTileRows);
    }

    // ---- stream
    if (c->opt.hip_stream) {
        c->stream = static_cast<hipStream_t>(c->opt.hip_stream);
    } else {
        HIPX(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    HIPX(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPX(hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
    HIPX(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    HIPX(hipEventCreate(&c->ev0));
    HIPX(hipEventCreate(&c->ev1));
    if (c->opt.output_ring_steps > 0) {
        HIPX(hipStreamCreateWithFlags(&c->out_stream, hipStreamNonBlocking));
        HIPX(hipEventCreateWithFlags(&c->out_ready, hipEventDisableTiming));
        HIPX(hipEventCreateWithFlags(&c->out_done, hipEventDisableTiming));
    }

    // ---- host staging of everything, then one copy each (Section 2.4.3)
    const int64_t S = c->stride;
    std::vector<float> h_state((size_t)INFOLI_NUM_STATE * S, 0.0f);
    std::vector<float> h_bias((size_t)S, 0.0f);
    std::vector<int64_t> h_rp((size_t)std::max<int64_t>(rp_total, 1));
    std::vector<int32_t> h_col((size_t)std::max<int64_t>(col_total, 1));
    std::vector<float> h_w((size_t)std::max<int64_t>(std::max(w_total, col_total), 1));
    std::vector<float> h_stream((size_t)std::max<int64_t>(stream_total, 1));
    std::vector<DevPulse> h_pulses((size_t)std::max(pulses_total, 1));
    bool any_cparams = false;
    for (int k = 0; k < ninst; ++k) any_cparams = any_cparams || specs[k].cell_params;
    std::vector<float> h_cparams(any_cparams ? (size_t)INFOLI_NUM_PARAMS * S : 1, 0.0f);
    for (int k = 0; k < ninst; ++k) {
        const infoli_network_spec& s = specs[k];
        const InstDesc& d = c->inst[k];
        const int64_t n = s.n_cells;
        float rest[INFOLI_NUM_STATE];
        rest_state_host(s.params ? s.params : kDefaultParams, -60.0f, rest);
        for (int64_t i = 0; i < n; ++i) {
            if (!s.init_state && s.cell_params)    // each cell's own rest state
                rest_state_host(s.cell_params + i * INFOLI_NUM_PARAMS, -60.0f, rest);
            for (int v = 0; v < INFOLI_NUM_STATE; ++v)
                h_state[v * S + d.cell_off + i] = s.init_state ? s.init_state[v * n + i] : rest[v];
        }
        if (s.cell_params)
            for (int v = 0; v < INFOLI_NUM_PARAMS; ++v)
                for (int64_t i = 0; i < n; ++i)
                    h_cparams[v * S + d.cell_off + i] = s.cell_params[i * INFOLI_NUM_PARAMS + v];
        if (s.i_bias)
            for (int64_t i = 0; i < n; ++i) h_bias[d.cell_off + i] = s.i_bias[i];
        if (s.conn == INFOLI_CONN_DENSE)
            std::memcpy(&h_w[d.w_off], s.w_dense, sizeof(float) * n * n);
        if (s.conn == INFOLI_CONN_CSR) {
            std::memcpy(&h_rp[d.rp_off], s.row_ptr, sizeof(int64_t) * (n + 1));
            if (s.nnz) std::memcpy(&h_col[d.w_off], s.col, sizeof(int32_t) * s.nnz);
            if (s.w_csr && s.nnz) std::memcpy(&h_w[d.w_off], s.w_csr, sizeof(float) * s.nnz);
        }
        for (int p = 0; p < s.n_pulses; ++p) {
            const infoli_pulse& q = s.pulses[p];
            DevPulse& dp = h_pulses[d.pulse_off + p];
            dp.n0 = q.step_begin;
            dp.n1 = q.step_end;
            dp.amp = q.amplitude;
            dp.c0 = q.cell_begin;
            dp.c1 = q.cell_end < 0 ? s.n_cells : q.cell_end;
            dp.pad0 = 0;
        }
        if (s.i_stream)
            std::memcpy(&h_stream[d.stream_off], s.i_stream, sizeof(float) * s.i_stream_steps * n);
    }

    c->state[0] = c->alloc<float>((size_t)INFOLI_NUM_STATE * S);
    c->state[1] = c->alloc<float>((size_t)INFOLI_NUM_STATE * S);
    c->igap = c->alloc<float>(S);
    c->bias = c->alloc<float>(S);
    c->d_inst = c->alloc<InstDesc>(ninst);
    c->d_pulses = c->alloc<DevPulse>(h_pulses.size());
    c->d_rowptr = c->alloc<int64_t>(h_rp.size());
    if (col16) {
        std::vector<uint16_t> h_c16(h_col.size());
        for (size_t e = 0; e < h_col.size(); ++e) h_c16[e] = (uint16_t)h_col[e];
        c->d_col16 = c->alloc<uint16_t>(h_c16.size());
        HIPX(hipMemcpy(c->d_col16, h_c16.data(), sizeof(uint16_t) * h_c16.size(), hipMemcpyHostToDevice));
        c->d_col = c->alloc<int32_t>(1);
    } else {
        c->d_col = c->alloc<int32_t>(h_col.size());
        c->d_col16 = c->alloc<uint16_t>(1);
    }
    c->d_w = c->alloc<float>(h_w.size());
    c->d_stream = c->alloc<float>(h_stream.size());
    c->d_spk_count = c->alloc<int32_t>(S);
    const int cap = c->opt.max_spikes_per_cell;
    c->d_spk_times = c->alloc<float>((size_t)S * std::max(cap, 1));
    c->d_flags = c->alloc<int32_t>(4);
    c->d_step = c->alloc<int64_t>(1);
    if (any_cparams) {
        c->d_cparams = c->alloc<float>(h_cparams.size());
        HIPX(hipMemcpy(c->d_cparams, h_cparams.data(), sizeof(float) * h_cparams.size(), hipMemcpyHostToDevice));
    }
    if (c->opt.output_ring_steps > 0) {
        c->out_slots = c->opt.output_ring_steps;
        c->out_ring = c->alloc<float>((size_t)c->out_slots * S);
        c->out_first = c->step;
    }

    HIPX(hipMemcpy(c->state[0], h_state.data(), sizeof(float) * h_state.size(), hipMemcpyHostToDevice));
    HIPX(hipMemcpy(c->state[1], h_state.data(), sizeof(float) * h_state.size(), hipMemcpyHostToDevice));
    HIPX(hipMemcpy(c->bias, h_bias.data(), sizeof(float) * S, hipMemcpyHostToDevice));
    HIPX(hipMemcpy(c->d_inst, c->inst.data(), sizeof(InstDesc) * ninst, hipMemcpyHostToDevice));
    HIPX(hipMemcpy(c->d_pulses, h_pulses.data(), sizeof(DevPulse) * h_pulses.size(), hipMemcpyHostToDevice));
    HIPX(hipMemcpy(c->d_rowptr, h_rp.data(), sizeof(int64_t) * h_rp.size(), hipMemcpyHostToDevice));
    if (!col16)
        HIPX(hipMemcpy(c->d_col, h_col.data(), sizeof(int32_t) * h_col.size(), hipMemcpyHostToDevice));
    HIPX(hipMemcpy(c->d_w, h_w.data(), sizeof(float) * h_w.size(), hipMemcpyHostToDevice));
    HIPX(hipMemcpy(c->d_stream, h_stream.data(), sizeof(float) * h_stream.size(), hipMemcpyHostToDevice));
    HIPX(hipMemset(c->d_spk_count, 0, sizeof(int32_t) * S));
    HIPX(hipMemset(c->d_spk_times, 0, sizeof(float) * (size_t)S * std::max(cap, 1)));
    HIPX(hipMemset(c->d_flags, 0, sizeof(int32_t) * 4));
    HIPX(hipMemset(c->igap, 0, sizeof(float) * S));
    HIPX(hipDeviceSynchronize());
    build_bitmaps(c, specs);
    build_blocks(c, specs);
    build_chunks(c, specs);
    build_sym(c);
    if (c->opt.autotune && c->opt.csr_path == 0) autotune(c);
    if (c->opt.csr_path == 3)
        for (int k = 0; k < ninst; ++k)
            if (c->inst[k].blk_off >= 0) {
                c->inst[k].blocked = 1;
                c->inst[k].lanes_per_row = std::min(64, std::max(8, c->inst[k].lanes_per_row));
                c->rows_of[k] = std::min(kMaxTileRows, 1024 / c->inst[k].lanes_per_row);
            }
    if (c->opt.csr_path == 4)
        for (int k = 0; k < ninst; ++k)
            if (c->inst[k].ca_off >= 0) c->inst[k].chunked = 1;
    if (c->opt.csr_path == 5)
        for (int k = 0; k < ninst; ++k)
            if (c->inst[k].cb_off >= 0 && !c->inst[k].has_w && !c->inst[k].pcell &&
                c->inst[k].nblk <= kStreamMaxBlocks && c->inst[k].cell_off % 4 == 0 && stream_ok(c)) {
                InstDesc d = c->inst[k];
                d.blocked = d.stream = 1;
                const int blk = c->opt.wide_threads ? c->opt.wide_threads : 1024;
                if (lds_floats_for(c, d, blk) * sizeof(float) + kStaticLds > (size_t)c->lds_max)
                    fail(INFOLI_E_UNSUPPORTED, "the chunk stream needs %zu bytes of LDS per workgroup, the device "
                         "gives %d", lds_floats_for(c, d, blk) * sizeof(float) + kStaticLds, c->lds_max);
                c->inst[k].blocked = c->inst[k].stream = 1;
                c->rows_of[k] = kSelfSlots;
            }
    if (c->opt.csr_path == 2)
        for (int k = 0; k < ninst; ++k)
            if (c->inst[k].bits_off >= 0) {
                c->inst[k].bitmap = 1;
                c->inst[k].wide = c->opt.wide_threads ? 1 : 0;   // in the wide group when its size is given
                c->rows_of[k] = kBitRows;
            }
    finalize_tiles(c);
    HIPX(hipDeviceSynchronize());
    if (persist_candidate && time_persistent_vs_tiles(c)) c->opt.step_mode = INFOLI_MODE_PERSISTENT;
}

}  // namespace

StepArgs infoli_rt::make_args(const infoli_ctx* c, bool device_step) {
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.inst = c->d_inst;
    a.tiles = c->grp[0].d_tiles;
    a.pulses = c->d_pulses;
    a.bias = c->bias;
    a.row_ptr = c->d_rowptr;
    a.col = c->d_col;
    a.col16 = c->d_col16;
    a.bits = c->d_bits;
    a.blk = c->d_blk;
    a.ca = c->d_ca;
    a.cb = c->d_cb;
    a.chk = c->d_chk;
    a.psym = c->d_psym;
    a.chkw = c->d_chkw;
    a.rtag = c->d_rtag;
    a.blk_cols = c->blk_cols;
    a.w = c->d_w;
    a.i_stream = c->d_stream;
    a.spike_count = c->d_spk_count;
    a.spike_times = c->d_spk_times;
    a.flags = c->d_flags;
    a.igap_out = c->igap;
    a.d_step = device_step ? c->d_step : nullptr;
    a.stride = c->stride;
    a.dt = c->dt;
    a.spike_cap = c->opt.max_spikes_per_cell;
    a.gap_only = 0;
    a.out_slots = c->out_slots;
    a.out_ring = c->out_ring;
    a.cparams = c->d_cparams;
    return a;
}

namespace {

hipGraphExec_t get_graph(infoli_ctx* c, int parity) {
    if (c->graph[parity]) return c->graph[parity];
    const StepArgs a = make_args(c, true);
    hipGraph_t g = nullptr;
    HIPX(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int from = parity;
    for (int k = 0; k < c->opt.graph_chunk; ++k) {
        launch_groups(c, c->cap_stream, a, from, 0, k, c->fork_groups);
        from ^= 1;
    }
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess) fail(INFOLI_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) fail(INFOLI_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    c->graph[parity] = ex;
    return ex;
}

void launch_persistent(infoli_ctx* c, int64_t n_steps, bool dry) {
    StepArgs a = make_args(c, false);
    a.dry = dry ? 1 : 0;
    const dim3 grid((unsigned)c->n_inst), block(kPersistBlock);
    const float* xin = c->state[c->cur];
    float* xout = c->state[c->cur ^ 1];
    switch (c->persist_cpt) {
        case 1: hipLaunchKernelGGL(k_persist<1>, grid, block, 0, c->stream, a, xin, xout, c->step, n_steps); break;
        case 2: hipLaunchKernelGGL(k_persist<2>, grid, block, 0, c->stream, a, xin, xout, c->step, n_steps); break;
        case 4: hipLaunchKernelGGL(k_persist<4>, grid, block, 0, c->stream, a, xin, xout, c->step, n_steps); break;
        default: hipLaunchKernelGGL(k_persist<8>, grid, block, 0, c->stream, a, xin, xout, c->step, n_steps); break;
    }
    if (dry) return;
    c->cur ^= 1;
    c->step += n_steps;
}

void run_steps(infoli_ctx* c, int64_t n_steps) {
    if (n_steps < 0) fail(INFOLI_E_INVALID_ARG, "n_steps must be >= 0");
    // steps that would overwrite ring slots of a queued output copy wait for it
    if (c->out_pending && c->step + n_steps - c->out_slots > c->out_pending_begin) {
        HIPX(hipStreamWaitEvent(c->stream, c->out_done, 0));
        c->out_pending = false;
    }
    HIPX(hipEventRecord(c->ev0, c->stream));
    int64_t left = n_steps;
    const int mode = c->opt.step_mode;
    if (mode == INFOLI_MODE_PERSISTENT) {
        if (left > 0) launch_persistent(c, left);
        left = 0;
    }
    const int64_t chunk = c->opt.graph_chunk;
    const bool use_graph = (mode == INFOLI_MODE_GRAPH) || (mode == INFOLI_MODE_AUTO && n_steps >= 2 * chunk);
    if (use_graph) {
        while (left >= chunk) {
            hipGraphExec_t ex = get_graph(c, c->cur);
            hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, c->stream, c->d_step, c->step);
            HIPX(hipGraphLaunch(ex, c->stream));
            c->step += chunk;
            left -= chunk;
        }
    }
    if (left > 0) {
        const StepArgs a = make_args(c, false);
        for (int64_t k = 0; k < left; ++k) {
            launch_groups(c, c->stream, a, c->cur, c->step, 0, false);
            c->cur ^= 1;
            c->step += 1;
        }
    }
    HIPX(hipGetLastError());
    HIPX(hipEventRecord(c->ev1, c->stream));
    c->timed = true;
}

}  // namespace

void infoli_rt::check_instance(const infoli_ctx* c, int32_t k) {
    if (k < 0 || k >= c->n_inst) fail(INFOLI_E_INVALID_ARG, "instance %d out of range", k);
}


extern "C" {

infoli_status infoli_default_options(infoli_options* opt) {
    if (!opt) {
        g_thread_error = "opt is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    std::memset(opt, 0, sizeof(*opt));
    opt->hip_stream = nullptr;
    opt->step_mode = INFOLI_MODE_AUTO;
    opt->graph_chunk = 100;
    opt->max_spikes_per_cell = 64;
    opt->tile_rows = 0;
    opt->lanes_per_row = 0;
    opt->check_finite = 1;
    opt->autotune = 1;
    return INFOLI_OK;
}

infoli_status infoli_default_params(float* out) {
    if (!out) {
        g_thread_error = "out is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    std::memcpy(out, kDefaultParams, sizeof(kDefaultParams));
    return INFOLI_OK;
}

infoli_status infoli_rest_state(const float* params, float v0_mv, float* out) {
    return guarded(nullptr, [&] {
        if (!out) fail(INFOLI_E_INVALID_ARG, "out is NULL");
        if (!std::isfinite(v0_mv)) fail(INFOLI_E_INVALID_ARG, "v0 not finite");
        if (params && !finite_all(params, INFOLI_NUM_PARAMS)) fail(INFOLI_E_INVALID_ARG, "non-finite parameter");
        rest_state_host(params ? params : kDefaultParams, v0_mv, out);
    });
}

infoli_status infoli_batch_init(const infoli_network_spec* specs, int32_t n_instances,
                                const infoli_options* opt, infoli_ctx** out) {
    if (!out) {
        g_thread_error = "out is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    *out = nullptr;
    infoli_ctx* c = new (std::nothrow) infoli_ctx();
    if (!c) {
        g_thread_error = "host allocation failed";
        return INFOLI_E_OUT_OF_MEMORY;
    }
    infoli_status st = guarded(nullptr, [&] {
        build_context(c, specs, n_instances, opt);
        // GRAPH mode: both captured chunks (by starting buffer) are built and
        // instantiated here, so no step call pays for capture
        if (c->opt.step_mode == INFOLI_MODE_GRAPH) {
            get_graph(c, 0);
            get_graph(c, 1);
        }
    });
    if (st != INFOLI_OK) {
        c->release();
        delete c;
        return st;
    }
    *out = c;
    return INFOLI_OK;
}

infoli_status infoli_init(const infoli_network_spec* spec, const infoli_options* opt, infoli_ctx** out) {
    return infoli_batch_init(spec, 1, opt, out);
}

infoli_status infoli_step(infoli_ctx* ctx, int64_t n_steps) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] { run_steps(ctx, n_steps); });
}

infoli_status infoli_sync(infoli_ctx* ctx) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        HIPX(hipStreamSynchronize(ctx->stream));
        if (ctx->opt.check_finite) {
            int32_t flag = 0;
            HIPX(hipMemcpy(&flag, ctx->d_flags, sizeof(flag), hipMemcpyDeviceToHost));
            if (flag) fail(INFOLI_E_NUMERIC, "a state value became NaN or infinite");
        }
    });
}

infoli_status infoli_read_state(infoli_ctx* ctx, int32_t instance, float* host_soa, int64_t cap_floats,
                                int64_t* step_out) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        check_instance(ctx, instance);
        const InstDesc& d = ctx->inst[instance];
        if (!host_soa) fail(INFOLI_E_INVALID_ARG, "host_soa is NULL");
        if (cap_floats < (int64_t)INFOLI_NUM_STATE * d.n)
            fail(INFOLI_E_INVALID_ARG, "capacity %lld < %lld", (long long)cap_floats,
                 (long long)INFOLI_NUM_STATE * d.n);
        HIPX(hipStreamSynchronize(ctx->stream));
        HIPX(hipMemcpy2D(host_soa, sizeof(float) * d.n, ctx->state[ctx->cur] + d.cell_off,
                         sizeof(float) * ctx->stride, sizeof(float) * d.n, INFOLI_NUM_STATE,
                         hipMemcpyDeviceToHost));
        if (step_out) *step_out = ctx->step;
    });
}

infoli_status infoli_read_state_device(infoli_ctx* ctx, int32_t instance, float* dev_soa) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        check_instance(ctx, instance);
        if (!dev_soa) fail(INFOLI_E_INVALID_ARG, "dev_soa is NULL");
        const InstDesc& d = ctx->inst[instance];
        HIPX(hipMemcpy2DAsync(dev_soa, sizeof(float) * d.n, ctx->state[ctx->cur] + d.cell_off,
                              sizeof(float) * ctx->stride, sizeof(float) * d.n, INFOLI_NUM_STATE,
                              hipMemcpyDeviceToDevice, ctx->stream));
    });
}

infoli_status infoli_write_state(infoli_ctx* ctx, int32_t instance, const float* host_soa, int64_t step) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        check_instance(ctx, instance);
        const InstDesc& d = ctx->inst[instance];
        if (!host_soa) fail(INFOLI_E_INVALID_ARG, "host_soa is NULL");
        if (step < 0) fail(INFOLI_E_INVALID_ARG, "step must be >= 0");
        if (!finite_all(host_soa, (int64_t)INFOLI_NUM_STATE * d.n))
            fail(INFOLI_E_INVALID_ARG, "non-finite state");
        HIPX(hipStreamSynchronize(ctx->stream));
        HIPX(hipMemcpy2D(ctx->state[ctx->cur] + d.cell_off, sizeof(float) * ctx->stride, host_soa,
                         sizeof(float) * d.n, sizeof(float) * d.n, INFOLI_NUM_STATE,
                         hipMemcpyHostToDevice));
        if (step != ctx->step && ctx->out_stream) {
            // a new step count: the ring's outputs belong to the old one
            HIPX(hipStreamSynchronize(ctx->out_stream));
            ctx->out_pending = false;
            ctx->out_first = step;
        }
        ctx->step = step;
    });
}

infoli_status infoli_read_gap_current(infoli_ctx* ctx, int32_t instance, float* host, int64_t cap) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        check_instance(ctx, instance);
        const InstDesc& d = ctx->inst[instance];
        if (!host) fail(INFOLI_E_INVALID_ARG, "host is NULL");
        if (cap < d.n) fail(INFOLI_E_INVALID_ARG, "capacity %lld < %d", (long long)cap, d.n);
        StepArgs a = make_args(ctx, false);
        a.gap_only = 1;
        launch_groups(ctx, ctx->stream, a, ctx->cur, ctx->step, 0, false);
        HIPX(hipGetLastError());
        HIPX(hipStreamSynchronize(ctx->stream));
        HIPX(hipMemcpy(host, ctx->igap + d.cell_off, sizeof(float) * d.n, hipMemcpyDeviceToHost));
    });
}

infoli_status infoli_read_spikes(infoli_ctx* ctx, int32_t instance, int32_t* counts, int64_t counts_cap,
                                 float* times_ms, int64_t times_cap) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        check_instance(ctx, instance);
        const InstDesc& d = ctx->inst[instance];
        const int cap = ctx->opt.max_spikes_per_cell;
        if (!counts) fail(INFOLI_E_INVALID_ARG, "counts is NULL");
        if (counts_cap < d.n) fail(INFOLI_E_INVALID_ARG, "counts capacity too small");
        if (times_ms && times_cap < (int64_t)d.n * cap) fail(INFOLI_E_INVALID_ARG, "times capacity too small");
        HIPX(hipStreamSynchronize(ctx->stream));
        HIPX(hipMemcpy(counts, ctx->d_spk_count + d.cell_off, sizeof(int32_t) * d.n, hipMemcpyDeviceToHost));
        if (times_ms && cap > 0)
            HIPX(hipMemcpy(times_ms, ctx->d_spk_times + d.cell_off * cap, sizeof(float) * d.n * cap,
                           hipMemcpyDeviceToHost));
    });
}

infoli_status infoli_output_copy_async(infoli_ctx* ctx, int64_t step_begin, int64_t n_steps, float* host,
                                       int64_t cap_floats) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        const int64_t R = ctx->out_slots;
        if (R == 0) fail(INFOLI_E_INVALID_ARG, "the context has no output ring (output_ring_steps = 0)");
        if (n_steps < 1 || n_steps > R) fail(INFOLI_E_INVALID_ARG, "n_steps must be in [1, %lld]", (long long)R);
        if (!host) fail(INFOLI_E_INVALID_ARG, "host is NULL");
        const int64_t cells = ctx->total_cells;
        if (cap_floats < n_steps * cells) fail(INFOLI_E_INVALID_ARG, "host capacity too small");
        if (step_begin + n_steps > ctx->step)
            fail(INFOLI_E_INVALID_ARG, "steps %lld..%lld are not queued yet (next step %lld)",
                 (long long)step_begin, (long long)(step_begin + n_steps - 1), (long long)ctx->step);
        if (step_begin < ctx->out_first || step_begin < ctx->step - R)
            fail(INFOLI_E_INVALID_ARG, "the output of step %lld is no longer in the ring", (long long)step_begin);
        HIPX(hipEventRecord(ctx->out_ready, ctx->stream));
        HIPX(hipStreamWaitEvent(ctx->out_stream, ctx->out_ready, 0));
        int64_t done = 0;
        while (done < n_steps) {
            const int64_t slot = (step_begin + done) % R;
            const int64_t len = std::min(n_steps - done, R - slot);
            HIPX(hipMemcpy2DAsync(host + done * cells, sizeof(float) * cells, ctx->out_ring + slot * ctx->stride,
                                  sizeof(float) * ctx->stride, sizeof(float) * cells, len, hipMemcpyDeviceToHost,
                                  ctx->out_stream));
            done += len;
        }
        HIPX(hipEventRecord(ctx->out_done, ctx->out_stream));
        if (!ctx->out_pending || step_begin < ctx->out_pending_begin) ctx->out_pending_begin = step_begin;
        ctx->out_pending = true;
    });
}

infoli_status infoli_output_wait(infoli_ctx* ctx) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        if (ctx->out_stream) HIPX(hipStreamSynchronize(ctx->out_stream));
    });
}

infoli_status infoli_clear_spikes(infoli_ctx* ctx) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        HIPX(hipStreamSynchronize(ctx->stream));
        HIPX(hipMemset(ctx->d_spk_count, 0, sizeof(int32_t) * ctx->stride));
        const int cap = std::max(ctx->opt.max_spikes_per_cell, 1);
        HIPX(hipMemset(ctx->d_spk_times, 0, sizeof(float) * ctx->stride * cap));
        HIPX(hipDeviceSynchronize());
    });
}

infoli_status infoli_get_info(const infoli_ctx* ctx, infoli_info* info) {
    if (!ctx || !info) {
        g_thread_error = "ctx or info is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    std::memset(info, 0, sizeof(*info));
    info->n_instances = ctx->n_inst;
    info->total_cells = ctx->total_cells;
    info->pairs_per_step = ctx->pairs_per_step;
    info->step = ctx->step;
    info->step_mode = ctx->opt.step_mode;
    info->n_tiles = (int32_t)tile_count(ctx);
    int32_t rows = 0, lanes = 0;
    for (int g = 0; g < 2; ++g)
        for (const Tile& t : ctx->grp[g].tiles) rows = std::max(rows, t.row1 - t.row0);
    for (const InstDesc& d : ctx->inst) lanes = std::max(lanes, d.lanes_per_row);
    info->tile_rows = rows;
    info->lanes_per_row = lanes;
    info->device_bytes = (int64_t)ctx->device_bytes;
    info->tuned = ctx->tuned;
    info->tune_cached = ctx->tune_cached;
    info->n_tiles_wide = (int32_t)ctx->grp[1].tiles.size();
    info->wide_threads = ctx->grp[1].block;
    info->tune_mode = ctx->tune_mode;
    for (const InstDesc& d : ctx->inst) {
        info->n_bitmap += d.conn == CONN_CSR && d.bitmap;
        info->n_blocked += d.conn == CONN_CSR && d.blocked;
        info->n_stream += d.conn == CONN_CSR && d.blocked && d.stream;
        if (d.conn == CONN_CSR && d.blocked && d.stream)
            info->stream_round = std::max(info->stream_round,
                                          d.stream_round >= 64 && d.stream_round <= kStreamRound ? d.stream_round
                                                                                                 : kStreamRound);
        info->n_sym += d.conn == CONN_UNIFORM && d.sym && ctx->opt.step_mode != INFOLI_MODE_PERSISTENT;
    }
    return INFOLI_OK;
}

infoli_status infoli_get_gap_path(const infoli_ctx* ctx, int32_t instance, int32_t* path, int32_t* vd_blocked) {
    if (!ctx) {
        g_thread_error = "ctx is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(const_cast<infoli_ctx*>(ctx), [&] {
        check_instance(ctx, instance);
        // the step kernel's own dispatch: the bitmap first; column blocks
        // only in the wide launch group (chunked when the block-major chunk
        // layout exists; simplified networks without it take row gathers);
        // else chunked rows or plain gathers
        const InstDesc& d = ctx->inst[instance];
        int32_t p = INFOLI_PATH_NONE, blk = 0;
        if (d.conn == CONN_UNIFORM)
            p = !d.sym || ctx->opt.step_mode == INFOLI_MODE_PERSISTENT ? INFOLI_PATH_UNIFORM
                : d.sgj                                                ? INFOLI_PATH_UNIFORM_SUM
                                                                       : INFOLI_PATH_UNIFORM_SYM;
        else if (d.conn == CONN_DENSE) p = INFOLI_PATH_DENSE;
        else if (d.conn == CONN_CSR) {
            const bool wide = ctx->group_of.size() > (size_t)instance && ctx->group_of[instance] == 1;
            if (ctx->opt.step_mode == INFOLI_MODE_PERSISTENT) p = INFOLI_PATH_CSR_GATHER;   // row walks
            else if (d.bitmap) p = INFOLI_PATH_CSR_BITMAP;
            else if (wide && d.blocked && d.stream && d.cb_off >= 0) p = INFOLI_PATH_CSR_STREAM, blk = 1;
            else if (wide && d.blocked && d.cb_off >= 0) p = INFOLI_PATH_CSR_CHUNKED, blk = 1;
            else if (wide && d.blocked && !d.sgj) p = INFOLI_PATH_CSR_GATHER, blk = 1;
            else p = d.chunked && d.ca_off >= 0 ? INFOLI_PATH_CSR_CHUNKED : INFOLI_PATH_CSR_GATHER;
        }
        if (path) *path = p;
        if (vd_blocked) *vd_blocked = blk;
    });
}

infoli_status infoli_last_step_ms(infoli_ctx* ctx, float* ms) {
    if (!ctx || !ms) {
        g_thread_error = "ctx or ms is NULL";
        return INFOLI_E_INVALID_ARG;
    }
    return guarded(ctx, [&] {
        if (!ctx->timed) fail(INFOLI_E_STATE, "no step has been timed yet");
        HIPX(hipEventSynchronize(ctx->ev1));
        HIPX(hipEventElapsedTime(ms, ctx->ev0, ctx->ev1));
    });
}

const char* infoli_state_var_name(int32_t v) {
    if (v < 0 || v >= INFOLI_NUM_STATE) return nullptr;
    return kStateNames[v];
}

const char* infoli_last_error(const infoli_ctx* ctx) {
    if (ctx) return ctx->err.c_str();
    return g_thread_error.c_str();
}

void infoli_destroy(infoli_ctx* ctx) {
    if (!ctx) return;
    try {
        ctx->release();
    } catch (...) {
    }
    delete ctx;
}

}  // extern "C"
