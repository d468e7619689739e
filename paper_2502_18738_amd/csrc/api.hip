// api.hip -- C ABI of libfiresim: validation, workspace carving, launch
// sequencing.  The contract of every entry point is documented in
// include/firesim.h.
#include "firesim.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMinTR = 8, kMinTC = 1;  // smallest whitelisted tile -> flag capacity
constexpr int kMaxN = 65536;
constexpr int kMaxSide = 1 << 16;
const float kC = 1.1486328125f;        // f_p constant of Eq. 5 / 8, FP32

thread_local std::string g_init_error;

size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct ScenLayout {
    int32_t pitch;
    int64_t PW;          // words per bit-plane
    int64_t max_tiles;   // flag capacity
    size_t rec, th8, q8, fuel, init, planes[2], flags[2], yhat, ckpt, tune, tign, tout;
};

struct Layout {
    size_t err, stats, box, part, jobs, tile_job, adj_jobs, adj_tile_job, sm8, lam,
        cell0, bl0, ib0, gpart_tmap, masks, adj_masks, tielog, tie_n, fbox, qbox, cell0q, qbits,
        total;
    int64_t qwords, max_qwords;       // block bit words: all scenarios, largest scenario
    std::vector<int64_t> qoff;        // first block bit word of each scenario
    int32_t mask_words, adj_mask_words;
    int64_t total_cells;
    int32_t tmap_blocks;
    int32_t max_h;
    std::vector<ScenLayout> s;
    std::vector<size_t> adj_planes[2], adj_flags[2];  // per (s, seg)
    int nseg;
    int64_t max_tiles_total, adj_max_tiles_total;
};

bool plan(const sim_desc* d, int n, uint32_t flags, int ckpt_every, int T_max, Layout* L) {
    const bool calib = flags & SIM_F_CALIB;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += up(bytes);
        return o;
    };
    L->s.assign(n, ScenLayout());
    L->nseg = calib ? (int)cdiv(T_max, ckpt_every) : 0;
    int64_t max_h = 0;
    L->err = take(64);
    L->stats = take(4 * sizeof(unsigned long long));
    L->tielog = L->tie_n = 0;
    if (flags & SIM_F_TIELOG) {
        L->tielog = take(sizeof(sim_tie) * (size_t)SIM_TIELOG_CAP);
        L->tie_n = take(sizeof(unsigned long long));
    }
    L->box = take(4 * sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) max_h = std::max<int64_t>(max_h, d[i].H);
    L->max_h = (int32_t)max_h;
    L->part = take(2 * sizeof(double) * (size_t)n * (size_t)cdiv(max_h, 4));
    L->jobs = take(sizeof(fs::DevScen) * (size_t)n);
    L->cell0 = take(sizeof(int64_t) * (size_t)(n + 1));
    L->ib0 = take(sizeof(int32_t) * (size_t)(n + 1));
    L->fbox = take(16 * (size_t)n);                     // burning box at the table's origin step
    L->qbox = take(16 * (size_t)n);                     // table region per scenario
    L->cell0q = take(sizeof(int64_t) * (size_t)(n + 1));
    // block bits of the table region (32 x 32-cell blocks, rows of
    // cdiv(pitch, 32) words): burning blocks, row-grown, grown
    L->qoff.assign(n + 1, 0);
    L->max_qwords = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t w = cdiv(d[i].H, 32) * cdiv(cdiv(d[i].W, 32), 32);
        L->qoff[i + 1] = L->qoff[i] + w;
        L->max_qwords = std::max(L->max_qwords, w);
    }
    L->qwords = L->qoff[n];
    L->qbits = take(3 * 4 * (size_t)L->qwords);
    L->total_cells = 0;
    for (int i = 0; i < n; ++i) L->total_cells += (int64_t)d[i].H * d[i].W;
    int64_t tiles = 0;
    for (int i = 0; i < n; ++i) {
        ScenLayout& s = L->s[i];
        s.pitch = (int32_t)cdiv(d[i].W, 32);
        s.PW = (int64_t)d[i].H * s.pitch;
        s.max_tiles = cdiv(d[i].H, kMinTR) * cdiv(s.pitch, kMinTC);
        tiles += s.max_tiles;
    }
    L->max_tiles_total = tiles;
    L->tile_job = take(sizeof(int32_t) * (size_t)tiles);
    L->mask_words = (int32_t)cdiv(tiles, 64);
    L->masks = take(3 * 8 * (size_t)L->mask_words);
    for (int i = 0; i < n; ++i) {
        ScenLayout& s = L->s[i];
        const int64_t cells = (int64_t)d[i].H * d[i].W;
        s.rec = take(16 * (size_t)cells);
        s.th8 = take(32 * (size_t)cells);
        s.q8 = take(32 * (size_t)cells);
        s.fuel = take(4 * (size_t)s.PW);
        s.init = take(4 * (size_t)s.PW);
        s.planes[0] = take(8 * (size_t)s.PW);
        s.planes[1] = take(8 * (size_t)s.PW);
        s.flags[0] = take((size_t)s.max_tiles);
        s.flags[1] = take((size_t)s.max_tiles);
        s.yhat = s.ckpt = s.tune = s.tign = s.tout = 0;
        if (!calib) s.tune = take(8 * (size_t)s.PW);   // state saved while autotuning
        if (calib) {
            s.yhat = take(4 * (size_t)cells);
            s.tign = take(4 * (size_t)cells);
            s.tout = take(4 * (size_t)cells);
            s.ckpt = take(8 * (size_t)s.PW * (size_t)L->nseg);
        }
    }
    L->adj_jobs = L->adj_tile_job = L->sm8 = L->lam = L->bl0 = L->gpart_tmap = 0;
    L->adj_masks = 0;
    L->adj_mask_words = 0;
    L->tmap_blocks = 0;
    L->adj_max_tiles_total = 0;
    for (int k = 0; k < 2; ++k) {
        L->adj_planes[k].clear();
        L->adj_flags[k].clear();
    }
    if (calib) {
        L->adj_jobs = take(sizeof(fs::DevScen) * (size_t)n * L->nseg);
        L->adj_max_tiles_total = tiles * L->nseg;
        L->adj_tile_job = take(sizeof(int32_t) * (size_t)L->adj_max_tiles_total);
        L->adj_mask_words = (int32_t)cdiv(L->adj_max_tiles_total, 64);
        L->adj_masks = take(3 * 8 * (size_t)L->adj_mask_words);
        int64_t cells = 0;
        for (int i = 0; i < n; ++i) cells += (int64_t)d[i].H * d[i].W;
        L->lam = take(4 * (size_t)cells);   // dL/dyhat of all scenarios, concatenated
        // burning-slot masks recorded by the checkpoint adjoint's recompute, one
        // byte per cell, concatenated like lam (cleared in 32-bit words)
        L->sm8 = take(4 * (size_t)cdiv(cells, 4));
        int64_t blocks = 0;
        for (int i = 0; i < n; ++i) blocks += cdiv((int64_t)d[i].H * d[i].W, 1024);   // gradient-pass segments
        L->tmap_blocks = (int32_t)blocks;
        L->bl0 = take(sizeof(int32_t) * (size_t)(n + 1));
        L->gpart_tmap = take(4 * sizeof(double) * (size_t)blocks);
        for (int i = 0; i < n; ++i)
            for (int g = 0; g < L->nseg; ++g)
                for (int k = 0; k < 2; ++k) {
                    L->adj_planes[k].push_back(take(8 * (size_t)L->s[i].PW));
                    L->adj_flags[k].push_back(take((size_t)L->s[i].max_tiles));
                }
    }
    L->total = off;
    return true;
}

bool finite_params(const sim_params& p) {
    return std::isfinite(p.p_h) && std::isfinite(p.a) && std::isfinite(p.c1) &&
           std::isfinite(p.c2) && std::isfinite(p.p_continue) && p.p_h >= 0.f &&
           p.p_continue >= 0.f && p.p_continue <= 1.f;
}

int check_descs(const sim_desc* d, int n, std::string* why) {
    if (!d) { *why = "descs is NULL"; return SIM_E_ARG; }
    if (n < 1 || n > kMaxN) { *why = "n out of range"; return SIM_E_SHAPE; }
    for (int i = 0; i < n; ++i) {
        char buf[160];
        if (d[i].H < 1 || d[i].W < 1 || d[i].H > kMaxSide || d[i].W > kMaxSide) {
            snprintf(buf, sizeof buf, "scenario %d: H, W must be in [1, %d]", i, kMaxSide);
            *why = buf;
            return SIM_E_SHAPE;
        }
        if (!(d[i].cell_m > 0.f) || !std::isfinite(d[i].cell_m)) {
            snprintf(buf, sizeof buf, "scenario %d: cell_m must be finite and > 0", i);
            *why = buf;
            return SIM_E_PARAM;
        }
        if (!finite_params(d[i].params)) {
            snprintf(buf, sizeof buf, "scenario %d: parameters must be finite, p_h >= 0, "
                     "0 <= p_continue <= 1", i);
            *why = buf;
            return SIM_E_PARAM;
        }
        const sim_fields& f = d[i].f;
        if (!f.p_veg || !f.p_den || !(f.elevation_m || f.slope_deg) || !f.init_burning) {
            snprintf(buf, sizeof buf, "scenario %d: a required field pointer is NULL", i);
            *why = buf;
            return SIM_E_ARG;
        }
        if (!f.wind_speed && (!std::isfinite(f.wind_speed_scalar) || f.wind_speed_scalar < 0.f)) {
            snprintf(buf, sizeof buf, "scenario %d: wind_speed_scalar must be finite, >= 0", i);
            *why = buf;
            return SIM_E_PARAM;
        }
        if (!f.wind_dir_deg && !std::isfinite(f.wind_dir_deg_scalar)) {
            snprintf(buf, sizeof buf, "scenario %d: wind_dir_deg_scalar must be finite", i);
            *why = buf;
            return SIM_E_PARAM;
        }
        if (((uintptr_t)f.p_veg | (uintptr_t)f.p_den | (uintptr_t)f.elevation_m |
             (uintptr_t)f.wind_speed | (uintptr_t)f.wind_dir_deg | (uintptr_t)f.slope_deg) & 3u) {
            snprintf(buf, sizeof buf, "scenario %d: FP32 fields must be 4-byte aligned", i);
            *why = buf;
            return SIM_E_ARG;
        }
    }
    return SIM_OK;
}

}  // namespace

struct sim_handle {
    int n = 0;
    uint32_t flags = 0;
    hipStream_t st = nullptr;
    int ckpt_every = 0, T_max = 0;
    std::vector<sim_desc> d;
    Layout L;
    char* ws = nullptr;
    std::vector<fs::DevScen> job;   // host mirror of the forward job table
    std::vector<int32_t> tile_job;
    int32_t ntiles = 0;
    std::vector<fs::DevScen> adj;   // adjoint jobs for the last run length
    std::vector<int32_t> adj_tile_job;
    int32_t adj_ntiles = 0, adj_T = -1;
    sim_exec ex{};
    fs::TileShape sh{};
    int parity = 0, step = 0;
    int lidx = 0;                   // launches since the worklist was last rebuilt
    int grid_max = 1024;            // work-groups of a worklist launch
    unsigned long long launches = 0;
    int64_t max_words = 0;
    std::string err;
    // captured launch sequences of sim_run, keyed by where they start
    struct Graph {
        int step, T, parity, ntiles, lmod;
        sim_exec ex;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    bool use_graphs = true;
    bool q_dirty = true;            // q8 tables must be rebuilt before the next step
    // The table covers the cells within (q_end - q_origin) of the burning box
    // taken at step q_origin: every ignition trial up to step q_end.
    int q_origin = 0, q_end = 0;
    // q_params: the parameters or the wind changed since the table was last
    // built; q_reset: the table's origin is the reset state (the same burning
    // cells after every reset), so a reset may keep a table built from it
    bool q_params = true, q_reset = false;
    // the parameters were last set on the device (sim_set_params_device): the
    // host copies in job[] and d[] are stale until pull_theta
    bool theta_dev = false;
    // calibration mode: the parameters changed after the run started, so the
    // checkpoints / time maps no longer match the parameters an adjoint would
    // differentiate; cleared by sim_reset
    bool stale = false;
    int adj_method = 0;             // 0: checkpoint recompute, 1: time maps
    fs::Rings rings{-1, 0, 0, 0};   // step-ring attach set (first < 0: every step)
    std::vector<int32_t> bl0;
    std::vector<int32_t> ib0;       // blocks of the state-reset kernel per scenario (prefix)
    std::vector<int64_t> cell0;
    hipStream_t cap = nullptr;      // private stream used only for capture
    int static_dev = -1;            // device whose static scratch this handle holds (-1: none)

    void drop_graphs() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
    ~sim_handle() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
    }

    fs::DevScen* d_jobs() { return reinterpret_cast<fs::DevScen*>(ws + L.jobs); }
    int32_t* d_tile_job() { return reinterpret_cast<int32_t*>(ws + L.tile_job); }
    int* d_err() { return reinterpret_cast<int*>(ws + L.err); }
    unsigned long long* d_stats() { return reinterpret_cast<unsigned long long*>(ws + L.stats); }
    unsigned long long* d_masks() { return reinterpret_cast<unsigned long long*>(ws + L.masks); }
    int4* d_fbox() { return reinterpret_cast<int4*>(ws + L.fbox); }
    bool calib() const { return flags & SIM_F_CALIB; }

    int fail(int code, const char* fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    int hip(hipError_t e, const char* what) {
        if (e == hipSuccess) return SIM_OK;
        return fail(SIM_E_HIP, "%s: %s", what, hipGetErrorString(e));
    }
};

namespace {

fs::TileShape shape_of(const sim_exec& e) {
    int km = 1;
    for (int k : {1, 4, 8, 16, 32})
        if (k >= e.depth) { km = k; break; }
    return fs::TileShape{e.tile_rows, e.tile_words, km, e.threads};
}

int refresh_worklist(sim_handle* h, bool dup);

// Bring parameters set on the device back into the host copies of the jobs
// (before the host copies are uploaded again).
int pull_theta(sim_handle* h) {
    if (!h->theta_dev) return SIM_OK;
    std::vector<fs::DevScen> dev((size_t)h->n);
    int rc = h->hip(hipMemcpyAsync(dev.data(), h->d_jobs(), sizeof(fs::DevScen) * h->n,
                                   hipMemcpyDeviceToHost, h->st), "read parameters");
    if (!rc) rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (rc) return rc;
    for (int i = 0; i < h->n; ++i) {
        fs::DevScen& J = h->job[i];
        J.p_h = dev[i].p_h;
        J.a = dev[i].a;
        J.c1 = dev[i].c1;
        J.c2 = dev[i].c2;
        h->d[i].params.p_h = J.p_h;
        h->d[i].params.a = J.a;
        h->d[i].params.c1 = J.c1;
        h->d[i].params.c2 = J.c2;
    }
    h->theta_dev = false;
    return SIM_OK;
}

// Recompute tile grids and the tile -> job table of the forward jobs.
int rebuild_tiles(sim_handle* h) {
    if (int rc = pull_theta(h)) return rc;
    int32_t g = 0;
    h->tile_job.clear();
    for (int i = 0; i < h->n; ++i) {
        fs::DevScen& J = h->job[i];
        J.tiles_r = (int32_t)cdiv(J.H, h->sh.tr);
        J.tiles_c = (int32_t)cdiv(J.pitch, h->sh.tc);
        J.tile0 = g;
        const int32_t nt = J.tiles_r * J.tiles_c;
        h->tile_job.insert(h->tile_job.end(), nt, i);
        g += nt;
    }
    h->ntiles = g;
    h->adj_T = -1;
    h->drop_graphs();
    int rc = h->hip(hipMemcpyAsync(h->d_jobs(), h->job.data(), sizeof(fs::DevScen) * h->n,
                                   hipMemcpyHostToDevice, h->st), "upload jobs");
    if (rc) return rc;
    rc = h->hip(hipMemcpyAsync(h->d_tile_job(), h->tile_job.data(), sizeof(int32_t) * g,
                               hipMemcpyHostToDevice, h->st), "upload tile table");
    if (rc) return rc;
    // the host vectors are reused by later calls: wait for the copies
    rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (rc) return rc;
    return refresh_worklist(h, true);
}

// After any change of the state or of the tiling: both ping-pong buffers
// equal to the current state, flags recomputed and the first worklist built.
int refresh_worklist(sim_handle* h, bool dup) {
    int rc = SIM_OK;
    if (dup)
        rc = h->hip(fs::launch_dup_planes(h->st, h->d_jobs(), h->n, h->parity, h->max_words),
                    "copy state");
    if (!rc) rc = h->hip(fs::launch_flags_init(h->st, h->d_jobs(), h->d_tile_job(), h->ntiles,
                                               h->parity, h->sh), "flags init");
    if (!rc) rc = h->hip(fs::launch_mask_init(h->st, h->d_jobs(), h->d_tile_job(), h->ntiles,
                                              h->parity, h->d_masks(), h->L.mask_words),
                         "worklist init");
    h->lidx = 0;
    return rc;
}

// The state changed other than by stepping (reset, set_state, spotting):
// the propagation table is rebuilt around the new burning box, unless this is
// a reset and the table was built around the reset state under the current
// parameters and wind (every reset starts from the same burning cells, so
// the region and every entry are those it would rebuild).
int take_origin(sim_handle* h, int origin_step, bool reset) {
    const bool keep = reset && h->q_reset && !h->q_params && !h->q_dirty;
    if (!keep) h->q_dirty = true;
    h->q_reset = reset;
    h->q_origin = origin_step;
    // a kept table needs no new burning box: the box and block bits of the
    // reset state it was built from are still in place (only this function
    // writes them, and the previous call was a reset as well), and a longer
    // run that grows the table reads them again
    if (keep) return SIM_OK;
    return h->hip(fs::launch_bbox(h->st, h->d_jobs(), h->n, h->parity, h->max_words, h->d_fbox(),
                                  reinterpret_cast<uint32_t*>(h->ws + h->L.qbits), h->L.qwords),
                  "burning box");
}

int save_ckpt(sim_handle* h, int slot) {
    return h->hip(fs::launch_ckpt_save(h->st, h->d_jobs(), h->n, h->parity, slot, h->max_words),
                  "checkpoint");
}

int reset_state(sim_handle* h) {
    h->parity = 0;
    h->step = 0;
    // the propagation table is rebuilt unless the last one was built around
    // the reset state with the current parameters and wind (take_origin)
    int rc = h->hip(fs::launch_init_state(h->st, h->d_jobs(),
                                          reinterpret_cast<const int32_t*>(h->ws + h->L.ib0),
                                          h->n, h->ib0.back(),
                                          reinterpret_cast<const int64_t*>(h->ws + h->L.cell0),
                                          h->L.total_cells, h->calib()), "init state");
    if (rc) return rc;
    rc = refresh_worklist(h, false);   // init_state wrote both buffers
    if (!rc) rc = take_origin(h, 0, true);
    if (rc) return rc;
    rc = h->hip(hipMemsetAsync(h->d_stats(), 0, 4 * sizeof(unsigned long long), h->st),
                "clear stats");
    if (!rc && (h->flags & SIM_F_TIELOG))
        rc = h->hip(hipMemsetAsync(h->ws + h->L.tie_n, 0, sizeof(unsigned long long), h->st),
                    "clear tie log");
    if (rc) return rc;
    h->launches = 0;
    if (h->calib()) return save_ckpt(h, 0);
    return SIM_OK;
}

}  // namespace

extern "C" {

const char* sim_version(void) { return "firesim 0.1 (gfx950)"; }

size_t sim_workspace_size(const sim_desc* descs, int32_t n, uint32_t flags, int32_t ckpt_every,
                          int32_t T_max) {
    std::string why;
    if (check_descs(descs, n, &why) != SIM_OK) return 0;
    if ((flags & SIM_F_CALIB) && (ckpt_every < 1 || T_max < 1)) return 0;
    Layout L;
    plan(descs, n, flags, ckpt_every, T_max, &L);
    return L.total;
}

}  // extern "C"

namespace {

// Checks shared by sim_init and sim_init_static (before any GPU work).
int check_init_args(sim_handle** out, const sim_desc* descs, int32_t n, uint32_t flags,
                    int32_t ckpt_every, int32_t T_max) {
    g_init_error.clear();
    if (!out) { g_init_error = "out is NULL"; return SIM_E_ARG; }
    *out = nullptr;
    std::string why;
    int rc = check_descs(descs, n, &why);
    if (rc) { g_init_error = why; return rc; }
    if (flags & ~(uint32_t)(SIM_F_CALIB | SIM_F_STATS | SIM_F_TIELOG)) {
        g_init_error = "unknown flag bits";
        return SIM_E_ARG;
    }
    if ((flags & SIM_F_CALIB) && (ckpt_every < 1 || T_max < 1)) {
        g_init_error = "calibration mode needs ckpt_every >= 1 and T_max >= 1";
        return SIM_E_SHAPE;
    }
    return SIM_OK;
}

// Handle set-up over a checked workspace (the caller's, or a device's static
// scratch): carves the workspace, builds the per-cell records, slope table,
// fuel plane and initial state, and reads the validation flag.
int init_handle(sim_handle** out, const sim_desc* descs, int32_t n, void* workspace,
                size_t ws_bytes, void* stream, uint32_t flags, int32_t ckpt_every,
                int32_t T_max) {
    int rc = SIM_OK;
    sim_handle* h = new (std::nothrow) sim_handle();
    if (!h) { g_init_error = "out of host memory"; return SIM_E_ARG; }
    h->n = n;
    h->flags = flags;
    h->st = (hipStream_t)stream;
    h->ckpt_every = (flags & SIM_F_CALIB) ? ckpt_every : 0;
    h->T_max = (flags & SIM_F_CALIB) ? T_max : 0;
    h->d.assign(descs, descs + n);
    plan(descs, n, flags, ckpt_every, T_max, &h->L);
    if (ws_bytes < h->L.total) {
        char buf[160];
        snprintf(buf, sizeof buf, "workspace too small: %zu < %zu bytes", ws_bytes, h->L.total);
        g_init_error = buf;
        delete h;
        return SIM_E_WORKSPACE;
    }
    h->ws = static_cast<char*>(workspace);

    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
            h->grid_max = 64 * cus;   // upper bound; occupancy decides the launch size
    }
    // default execution shape
    int32_t max_pitch = 0;
    for (const auto& s : h->L.s) max_pitch = std::max(max_pitch, s.pitch);
    h->ex = sim_exec{32, 2, 32, 1, 0};
    (void)max_pitch;
    h->sh = shape_of(h->ex);

    h->job.resize(n);
    for (int i = 0; i < n; ++i) {
        const sim_desc& d = descs[i];
        const ScenLayout& s = h->L.s[i];
        fs::DevScen& J = h->job[i];
        std::memset(&J, 0, sizeof J);
        J.H = d.H;
        J.W = d.W;
        J.pitch = s.pitch;
        J.sidx = i;
        if (flags & SIM_F_TIELOG) {
            J.tielog = h->ws + h->L.tielog;
            J.tie_n = reinterpret_cast<unsigned long long*>(h->ws + h->L.tie_n);
        }
        J.t_base = 0;
        J.t_end = INT_MAX;
        J.scen_id = d.scenario_id;
        J.seed_lo = (uint32_t)d.seed;
        J.seed_hi = (uint32_t)(d.seed >> 32);
        J.inv_l = 1.0f / d.cell_m;
        J.inv_l_diag = (float)(1.0 / (std::sqrt(2.0) * (double)d.cell_m));
        J.p_h = d.params.p_h;
        J.a = d.params.a;
        J.c1 = d.params.c1;
        J.c2 = d.params.c2;
        J.p_continue = d.params.p_continue;
        J.c = kC;
        J.elev = d.f.elevation_m;
        J.rec = reinterpret_cast<const float4*>(h->ws + s.rec);
        J.th8 = reinterpret_cast<const float*>(h->ws + s.th8);
        J.q8 = reinterpret_cast<float*>(h->ws + s.q8);
        J.init = reinterpret_cast<const uint32_t*>(h->ws + s.init);
        J.fuel = reinterpret_cast<const uint32_t*>(h->ws + s.fuel);
        J.planes[0] = reinterpret_cast<uint32_t*>(h->ws + s.planes[0]);
        J.planes[1] = reinterpret_cast<uint32_t*>(h->ws + s.planes[1]);
        J.flags[0] = reinterpret_cast<uint8_t*>(h->ws + s.flags[0]);
        J.flags[1] = reinterpret_cast<uint8_t*>(h->ws + s.flags[1]);
        J.yhat = h->calib() ? reinterpret_cast<float*>(h->ws + s.yhat) : nullptr;
        J.tign = h->calib() ? reinterpret_cast<int32_t*>(h->ws + s.tign) : nullptr;
        J.tout = h->calib() ? reinterpret_cast<int32_t*>(h->ws + s.tout) : nullptr;
        J.ckpt = h->calib() ? reinterpret_cast<uint32_t*>(h->ws + s.ckpt) : nullptr;
        J.sm8 = nullptr;   // set below with lam_off
        uint32_t* qb = reinterpret_cast<uint32_t*>(h->ws + h->L.qbits);
        J.qburn = qb + h->L.qoff[i];
        J.qrow = qb + h->L.qwords + h->L.qoff[i];
        J.qneed = qb + 2 * h->L.qwords + h->L.qoff[i];
        J.lam_off = 0;   // set below: offset of this scenario's grid in dL/dyhat
        h->max_words = std::max<int64_t>(h->max_words, s.PW);
    }

    // error flag and count of rejected device parameter rows
    rc = h->hip(hipMemsetAsync(h->d_err(), 0, 2 * sizeof(int), h->st), "clear error flag");
    for (int i = 0; i < n && !rc; ++i) {
        const sim_desc& d = descs[i];
        fs::DevScen& J = h->job[i];
        rc = h->hip(fs::launch_prologue(h->st, nullptr, J, d.f.p_veg, d.f.p_den, d.f.wind_speed,
                                        d.f.wind_dir_deg, d.f.wind_speed_scalar,
                                        d.f.wind_dir_deg_scalar, d.f.init_burning,
                                        const_cast<float4*>(J.rec),
                                        const_cast<uint32_t*>(J.fuel), J.yhat, h->d_err()),
                    "prologue");
    }
    for (int i = 0; i < n && !rc; ++i)
        rc = h->hip(fs::launch_slopes(h->st, h->job[i], const_cast<float*>(h->job[i].th8),
                                      descs[i].f.slope_deg, h->d_err()), "slope table");
    // Table entries outside the region a run can reach are never read; they
    // start as NaN, so that a read outside the region (a defect) could only
    // make p_ignite NaN and the trial fail visibly, never pass silently.
    for (int i = 0; i < n && !rc; ++i)
        rc = h->hip(fs::launch_fill_u32(h->st, reinterpret_cast<uint32_t*>(h->job[i].q8),
                                        (size_t)8 * descs[i].H * descs[i].W, 0x7FC00000u),
                    "table fill");
    // keep the packed initial burning plane for every reset
    for (int i = 0; i < n && !rc; ++i)
        rc = h->hip(hipMemcpyAsync(const_cast<uint32_t*>(h->job[i].init), h->job[i].planes[0],
                                   4 * (size_t)h->L.s[i].PW, hipMemcpyDeviceToDevice, h->st),
                    "keep initial state");
    h->cell0.assign(1, 0);
    for (int i = 0; i < n; ++i) h->cell0.push_back(h->cell0.back() + (int64_t)descs[i].H * descs[i].W);
    for (int i = 0; i < n; ++i) {
        h->job[i].lam_off = h->cell0[i];
        if (h->calib()) h->job[i].sm8 = reinterpret_cast<uint8_t*>(h->ws + h->L.sm8) + h->cell0[i];
    }
    if (!rc) rc = h->hip(hipMemcpyAsync(h->ws + h->L.cell0, h->cell0.data(),
                                        sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, h->st),
                         "upload cell offsets");
    h->ib0.assign(1, 0);
    for (int i = 0; i < n; ++i)
        h->ib0.push_back(h->ib0.back() + (int32_t)cdiv(h->L.s[i].PW, 1024));   // 4 words per lane
    if (!rc) rc = h->hip(hipMemcpyAsync(h->ws + h->L.ib0, h->ib0.data(), sizeof(int32_t) * (n + 1),
                                        hipMemcpyHostToDevice, h->st), "upload reset blocks");
    if (!rc && h->calib()) {
        h->bl0.assign(1, 0);
        for (int i = 0; i < n; ++i)
            h->bl0.push_back(h->bl0.back() + (int32_t)cdiv((int64_t)descs[i].H * descs[i].W, 1024));
        rc = h->hip(hipMemcpyAsync(h->ws + h->L.bl0, h->bl0.data(), sizeof(int32_t) * (n + 1),
                                   hipMemcpyHostToDevice, h->st), "upload block offsets");
    }
    if (!rc) rc = rebuild_tiles(h);   // synchronises the stream
    if (!rc) rc = reset_state(h);
    int bad = 0;
    if (!rc) rc = h->hip(hipMemcpyAsync(&bad, h->d_err(), sizeof(int), hipMemcpyDeviceToHost,
                                        h->st), "read validation flag");
    if (!rc) rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (!rc && bad) {
        std::string m = "invalid field values:";
        if (bad & 1) m += " p_veg < -1 or non-finite;";
        if (bad & 2) m += " p_den < -1 or non-finite;";
        if (bad & 4) m += " non-finite elevation;";
        if (bad & 8) m += " wind speed < 0 or non-finite;";
        if (bad & 16) m += " non-finite wind direction;";
        if (bad & 64) m += " non-finite slope_deg entry;";
        g_init_error = m;
        delete h;
        return SIM_E_PARAM;
    }
    if (rc) {
        g_init_error = h->err;
        delete h;
        return rc;
    }
    *out = h;
    return SIM_OK;
}

// Scratch of sim_init_static: the workspace of the one static handle a device
// may hold at a time.  In host code `scratch` names a host-side stand-in, not
// device memory: every host use goes through the per-device address that
// hipGetSymbolAddress returns (g_static.ptr), never through the name.
constexpr size_t kStaticScratchBytes = SIM_STATIC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
struct StaticSlots {
    std::mutex mu;
    void* ptr[kMaxDevices] = {};      // device address of `scratch` on each device
    bool held[kMaxDevices] = {};      // a live static handle uses that device's array
} g_static;

void release_static(sim_handle* h) {
    if (!h || h->static_dev < 0) return;
    std::lock_guard<std::mutex> lk(g_static.mu);
    g_static.held[h->static_dev] = false;
    h->static_dev = -1;
}

}  // namespace

extern "C" {

int sim_init(sim_handle** out, const sim_desc* descs, int32_t n, void* workspace,
             size_t ws_bytes, void* stream, uint32_t flags, int32_t ckpt_every, int32_t T_max) {
    int rc = check_init_args(out, descs, n, flags, ckpt_every, T_max);
    if (rc) return rc;
    if (!workspace) { g_init_error = "workspace is NULL"; return SIM_E_ARG; }
    if ((uintptr_t)workspace % kAlign) {
        g_init_error = "workspace must be 256-byte aligned";
        return SIM_E_WORKSPACE;
    }
    return init_handle(out, descs, n, workspace, ws_bytes, stream, flags, ckpt_every, T_max);
}

int sim_init_static(sim_handle** out, const sim_desc* descs, int32_t n, void* stream,
                    uint32_t flags, int32_t ckpt_every, int32_t T_max) {
    int rc = check_init_args(out, descs, n, flags, ckpt_every, T_max);
    if (rc) return rc;
    Layout L;
    plan(descs, n, flags, ckpt_every, T_max, &L);
    if (L.total > kStaticScratchBytes) {
        char buf[200];
        snprintf(buf, sizeof buf, "these scenarios need %zu bytes of workspace; the static "
                 "scratch holds %zu (use sim_init with a workspace)", L.total,
                 kStaticScratchBytes);
        g_init_error = buf;
        return SIM_E_WORKSPACE;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        g_init_error = "no current HIP device (or device index >= 64)";
        return SIM_E_HIP;
    }
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static.mu);
        if (g_static.held[dev]) {
            g_init_error = "the static scratch of this device is held by another handle "
                           "(sim_destroy it first)";
            return SIM_E_STATE;
        }
        if (!g_static.ptr[dev]) {
            // once per device, with that device current: the address of this
            // device's copy of the array
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                g_init_error = std::string("hipGetSymbolAddress(scratch): ") +
                               hipGetErrorString(e);
                return SIM_E_HIP;
            }
            if ((uintptr_t)p % kAlign) {
                g_init_error = "static scratch is not 256-byte aligned";
                return SIM_E_WORKSPACE;
            }
            g_static.ptr[dev] = p;
        }
        ws = g_static.ptr[dev];
        g_static.held[dev] = true;
    }
    rc = init_handle(out, descs, n, ws, kStaticScratchBytes, stream, flags, ckpt_every, T_max);
    if (rc) {
        std::lock_guard<std::mutex> lk(g_static.mu);
        g_static.held[dev] = false;
        return rc;
    }
    (*out)->static_dev = dev;
    return SIM_OK;
}

int sim_set_exec(sim_handle* h, const sim_exec* e) {
    if (!h || !e) return h ? h->fail(SIM_E_ARG, "exec is NULL") : SIM_E_ARG;
    if (e->depth < 1 || e->depth > 32 || e->depth > e->tile_rows)
        return h->fail(SIM_E_SHAPE, "depth must be in [1, min(32, tile_rows)]");
    const fs::TileShape sh = shape_of(*e);
    if (!fs::step_shape_supported(sh, false) ||
        (h->calib() && !fs::step_shape_supported(sh, true)))
        return h->fail(SIM_E_SHAPE, "tile %dx%d words with depth %d (%d threads) is not compiled in",
                       e->tile_rows, e->tile_words, e->depth, e->threads);
    if (e->skip < 0 || e->skip > 3) return h->fail(SIM_E_ARG, "skip must be 0, 1, 2 or 3");
    h->ex = *e;
    const bool same = sh.tr == h->sh.tr && sh.tc == h->sh.tc;
    h->sh = sh;
    if (same) return refresh_worklist(h, true);
    return rebuild_tiles(h);
}

int sim_get_exec(const sim_handle* h, sim_exec* e) {
    if (!h || !e) return SIM_E_ARG;
    *e = h->ex;
    return SIM_OK;
}

}  // extern "C"

namespace {

// Enqueue the launches of T steps on `st`, advancing the handle's counters.
int enqueue_run(sim_handle* h, hipStream_t st, int T, unsigned long long* stats) {
    while (T > 0) {
        int k = std::min(h->ex.depth, T);
        if (h->calib()) k = std::min(k, h->ckpt_every - h->step % h->ckpt_every);
        fs::Sched sc{nullptr, nullptr, nullptr, h->L.mask_words};
        if (h->ex.skip == 1 || h->ex.skip == 3) {
            unsigned long long* m = h->d_masks();
            const int64_t nw = h->L.mask_words;
            sc.in = m + nw * (h->lidx % 3);
            sc.out = m + nw * ((h->lidx + 1) % 3);
            sc.clear = m + nw * ((h->lidx + 2) % 3);
        }
        // (launches over every tile of a single scenario need no tile -> job table)
        int rc = h->hip(fs::launch_step(st, h->sh, false, h->d_jobs(),
                                        h->n == 1 && h->ex.skip != 1 ? nullptr : h->d_tile_job(),
                                        h->ntiles,
                                        h->parity, h->step, k, h->ex.skip, nullptr,
                                        fs::Rings{-1, 0, 0, 0}, sc, h->grid_max, stats),
                        "step kernel");
        ++h->lidx;
        if (rc) return rc;
        ++h->launches;
        h->parity ^= 1;
        h->step += k;
        T -= k;
        if (h->calib() && h->step % h->ckpt_every == 0 && h->step < h->T_max) {
            rc = h->hip(fs::launch_ckpt_save(st, h->d_jobs(), h->n, h->parity,
                                             h->step / h->ckpt_every, h->max_words),
                        "checkpoint");
            if (rc) return rc;
        }
    }
    return SIM_OK;
}

// Make the per-edge propagation table (Eq. 2-5 for every edge) valid for
// every ignition trial up to step t_end: rebuilt when the parameters, the
// wind or the state's origin changed, or when t_end passes the steps it was
// built for.  It covers the cells within t_end - q_origin of the burning box
// at step q_origin: fire moves at most one cell per step, so a cell with a
// burning neighbour at step t - 1 <= t_end - 1 lies within t - q_origin of it.
int ensure_qtable(sim_handle* h, int64_t t_end) {
    if (!h->q_dirty && t_end <= h->q_end) return SIM_OK;
    const int reach = (int)std::min<int64_t>(std::max<int64_t>(t_end - h->q_origin, 0), kMaxSide);
    int rc = h->hip(fs::launch_qtable(h->st, h->d_jobs(), h->d_fbox(), h->n, reach,
                                      h->L.total_cells, h->L.max_qwords,
                                      reinterpret_cast<int4*>(h->ws + h->L.qbox),
                                      reinterpret_cast<int64_t*>(h->ws + h->L.cell0q)),
                    "propagation table");
    if (!rc) {
        h->q_dirty = h->q_params = false;
        h->q_end = (int)std::min<int64_t>(t_end, INT_MAX);
    }
    return rc;
}

bool same_exec(const sim_exec& a, const sim_exec& b) {
    return a.tile_rows == b.tile_rows && a.tile_words == b.tile_words && a.depth == b.depth &&
           a.skip == b.skip && a.threads == b.threads;
}

// Replay (or capture, then replay) the launch sequence of T steps from the
// handle's current step and parity as one HIP graph on the handle's stream.
// Returns SIM_E_STATE when capture is not possible (the caller then launches
// directly).
int run_graph(sim_handle* h, int T) {
    for (auto& g : h->graphs) {
        if (g.step == h->step && g.T == T && g.parity == h->parity && g.ntiles == h->ntiles &&
            g.lmod == h->lidx % 3 && same_exec(g.ex, h->ex)) {
            int rc = h->hip(hipGraphLaunch(g.exec, h->st), "graph launch");
            if (rc) return rc;
            // advance the counters exactly as the captured sequence did
            int t = T, st = h->step, par = h->parity;
            while (t > 0) {
                int k = std::min(h->ex.depth, t);
                if (h->calib()) k = std::min(k, h->ckpt_every - st % h->ckpt_every);
                par ^= 1;
                st += k;
                t -= k;
                ++h->launches;
                ++h->lidx;
            }
            h->step = st;
            h->parity = par;
            return SIM_OK;
        }
    }
    if (!h->cap && hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) {
        h->cap = nullptr;
        return SIM_E_STATE;
    }
    const int step0 = h->step, par0 = h->parity, lidx0 = h->lidx;
    const unsigned long long l0 = h->launches;
    if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return SIM_E_STATE;
    int rc = enqueue_run(h, h->cap, T, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap, &graph);
    hipGraphExec_t exec = nullptr;
    if (!rc && e == hipSuccess && graph &&
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
        (void)hipGraphDestroy(graph);
        if (h->graphs.size() >= 8) {
            (void)hipGraphExecDestroy(h->graphs.front().exec);
            h->graphs.erase(h->graphs.begin());
        }
        h->graphs.push_back(sim_handle::Graph{step0, T, par0, h->ntiles, lidx0 % 3, h->ex, exec});
        return h->hip(hipGraphLaunch(exec, h->st), "graph launch");
    }
    if (graph) (void)hipGraphDestroy(graph);
    // capture failed: undo the counter updates, let the caller launch directly
    h->step = step0;
    h->parity = par0;
    h->lidx = lidx0;
    h->launches = l0;
    h->use_graphs = false;
    return SIM_E_STATE;
}

}  // namespace

extern "C" {

int sim_run(sim_handle* h, int32_t T) {
    if (!h) return SIM_E_ARG;
    if (T < 0) return h->fail(SIM_E_SHAPE, "T must be >= 0");
    if (h->calib() && (int64_t)h->step + T > h->T_max)
        return h->fail(SIM_E_STATE, "calibration run would pass T_max = %d", h->T_max);
    if ((int64_t)h->step + T > INT_MAX / 2) return h->fail(SIM_E_SHAPE, "step counter overflow");
    if (T == 0) return SIM_OK;
    int qrc = ensure_qtable(h, (int64_t)h->step + T);
    if (qrc) return qrc;
    unsigned long long* stats = (h->flags & SIM_F_STATS) ? h->d_stats() : nullptr;
    if (h->use_graphs && !stats && T > h->ex.depth) {
        const int rc = run_graph(h, T);
        if (rc != SIM_E_STATE) return rc;
    }
    return enqueue_run(h, h->st, T, stats);
}

int sim_prepare(sim_handle* h, int32_t T) {
    if (!h) return SIM_E_ARG;
    if (T < 0) return h->fail(SIM_E_SHAPE, "T must be >= 0");
    return ensure_qtable(h, (int64_t)h->step + T);
}

int sim_autotune(sim_handle* h, int32_t T_probe, sim_exec* best) {
    if (!h) return SIM_E_ARG;
    if (h->calib()) return h->fail(SIM_E_STATE, "sim_autotune is not available in calibration mode");
    if (T_probe < 1 || T_probe > 4096) return h->fail(SIM_E_SHAPE, "T_probe must be in [1, 4096]");
    fs::TileShape shapes[64];
    const int ns = fs::step_shapes(shapes, 64);
    if (int r = ensure_qtable(h, (int64_t)h->step + T_probe)) return r;
    const int step0 = h->step, par0 = h->parity;
    const sim_exec ex0 = h->ex;
    int rc = SIM_OK;
    for (int i = 0; i < h->n && !rc; ++i)
        rc = h->hip(hipMemcpyAsync(h->ws + h->L.s[i].tune, h->job[i].planes[par0],
                                   8 * (size_t)h->L.s[i].PW, hipMemcpyDeviceToDevice, h->st),
                    "save state");
    if (rc) return rc;
    auto restore = [&]() -> int {
        for (int i = 0; i < h->n; ++i) {
            int r = h->hip(hipMemcpyAsync(h->job[i].planes[0], h->ws + h->L.s[i].tune,
                                          8 * (size_t)h->L.s[i].PW, hipMemcpyDeviceToDevice,
                                          h->st), "restore state");
            if (r) return r;
        }
        h->parity = 0;
        h->step = step0;
        return refresh_worklist(h, true);
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return h->fail(SIM_E_HIP, "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return h->fail(SIM_E_HIP, "event create");
    }
    const bool graphs = h->use_graphs;
    h->use_graphs = false;
    float best_ms = 1e30f;
    sim_exec best_ex = ex0;
    for (int c = 0; c < 3 * ns && !rc; ++c) {
        // the probe's steps in as few launches as the halo allows, spread
        // evenly over them (20 steps on a 16-step halo: two launches of 10,
        // whose cells need 10 halo rows, not 16)
        const int km = shapes[c % ns].km;
        const int launches = (T_probe + km - 1) / km;
        sim_exec ex{shapes[c % ns].tr, shapes[c % ns].tc,
                    std::min(km, (T_probe + launches - 1) / launches), 1 + c / ns,
                    shapes[c % ns].nt};
        // (a depth that maps to a smaller halo would select another, possibly
        // uncompiled shape: such short probes keep the shape's own halo)
        if (shape_of(ex).km != km) ex.depth = km;
        rc = sim_set_exec(h, &ex);
        if (!rc) rc = restore();
        if (!rc) rc = enqueue_run(h, h->st, T_probe, nullptr);   // warm-up
        if (!rc) rc = restore();
        if (!rc) rc = h->hip(hipEventRecord(e0, h->st), "event record");
        if (!rc) rc = enqueue_run(h, h->st, T_probe, nullptr);
        if (!rc) rc = h->hip(hipEventRecord(e1, h->st), "event record");
        if (!rc) rc = h->hip(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        if (!rc) rc = h->hip(hipEventElapsedTime(&ms, e0, e1), "elapsed time");
        if (!rc && ms < best_ms) {
            best_ms = ms;
            best_ex = ex;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->use_graphs = graphs;
    if (!rc) rc = sim_set_exec(h, &best_ex);
    if (!rc) rc = restore();
    if (!rc) h->parity = 0;
    if (!rc && best) *best = best_ex;
    return rc;
}

int sim_use_graphs(sim_handle* h, int32_t on) {
    if (!h) return SIM_E_ARG;
    h->use_graphs = on != 0;
    if (!on) h->drop_graphs();
    return SIM_OK;
}

int sim_step(sim_handle* h) { return sim_run(h, 1); }

int sim_get_step(const sim_handle* h, int32_t* step) {
    if (!h || !step) return SIM_E_ARG;
    *step = h->step;
    return SIM_OK;
}

int sim_set_params(sim_handle* h, const sim_params* p) {
    if (!h) return SIM_E_ARG;
    if (!p) return h->fail(SIM_E_ARG, "params is NULL");
    for (int i = 0; i < h->n; ++i)
        if (!finite_params(p[i]))
            return h->fail(SIM_E_PARAM, "scenario %d: parameters must be finite, p_h >= 0, "
                           "0 <= p_continue <= 1", i);
    for (int first = 0; first < h->n; first += 64) {
        fs::ParamBlock pb;
        pb.first = first;
        pb.count = std::min(64, h->n - first);
        for (int i = 0; i < pb.count; ++i) {
            const sim_params& q = p[first + i];
            pb.v[i][0] = q.p_h;
            pb.v[i][1] = q.a;
            pb.v[i][2] = q.c1;
            pb.v[i][3] = q.c2;
            pb.v[i][4] = q.p_continue;
            fs::DevScen& J = h->job[first + i];
            J.p_h = q.p_h;
            J.a = q.a;
            J.c1 = q.c1;
            J.c2 = q.c2;
            J.p_continue = q.p_continue;
            h->d[first + i].params = q;
        }
        int rc = h->hip(fs::launch_set_params(h->st, h->d_jobs(), pb), "set params");
        if (rc) return rc;
    }
    // (the adjoint's segment jobs take the new parameters on the device before
    // their next recompute)
    h->theta_dev = false;
    h->q_dirty = h->q_params = true;
    if (h->calib() && h->step != 0) h->stale = true;
    return SIM_OK;
}

int sim_set_params_device(sim_handle* h, const float* theta) {
    if (!h) return SIM_E_ARG;
    if (!theta) return h->fail(SIM_E_ARG, "theta is NULL");
    if ((uintptr_t)theta & 3u) return h->fail(SIM_E_ARG, "theta must be 4-byte aligned");
    int rc = h->hip(fs::launch_set_theta(h->st, h->d_jobs(), h->n, theta, h->d_err() + 1),
                    "set parameters on the device");
    if (rc) return rc;
    h->theta_dev = true;
    h->q_dirty = h->q_params = true;
    if (h->calib() && h->step != 0) h->stale = true;
    return SIM_OK;
}

int sim_params_rejected(sim_handle* h, int32_t* count) {
    if (!h) return SIM_E_ARG;
    if (!count) return h->fail(SIM_E_ARG, "count is NULL");
    int v = 0;
    int rc = h->hip(hipMemcpyAsync(&v, h->d_err() + 1, sizeof(int), hipMemcpyDeviceToHost,
                                   h->st), "read rejected count");
    if (!rc) rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (!rc) rc = h->hip(hipMemsetAsync(h->d_err() + 1, 0, sizeof(int), h->st),
                         "clear rejected count");
    if (!rc) *count = v;
    return rc;
}

int sim_reset(sim_handle* h, const uint64_t* seeds) {
    if (!h) return SIM_E_ARG;
    if (seeds) {
        for (int first = 0; first < h->n; first += 64) {
            fs::SeedBlock sb;
            sb.first = first;
            sb.count = std::min(64, h->n - first);
            for (int i = 0; i < sb.count; ++i) {
                sb.lo[i] = (uint32_t)seeds[first + i];
                sb.hi[i] = (uint32_t)(seeds[first + i] >> 32);
                h->job[first + i].seed_lo = sb.lo[i];
                h->job[first + i].seed_hi = sb.hi[i];
                h->d[first + i].seed = seeds[first + i];
            }
            int rc = h->hip(fs::launch_set_seeds(h->st, h->d_jobs(), sb), "set seeds");
            if (rc) return rc;
        }
    }
    h->stale = false;
    return reset_state(h);
}

int sim_get_state(sim_handle* h, int32_t s, uint8_t* out) {
    if (!h) return SIM_E_ARG;
    if (s < 0 || s >= h->n) return h->fail(SIM_E_ARG, "scenario index %d out of range", s);
    if (!out) return h->fail(SIM_E_ARG, "out is NULL");
    const fs::DevScen& J = h->job[s];
    return h->hip(fs::launch_get_state(h->st, J, J.planes[h->parity], out), "get state");
}

int sim_set_state(sim_handle* h, int32_t s, const uint8_t* in, int32_t step) {
    if (!h) return SIM_E_ARG;
    if (s < 0 || s >= h->n) return h->fail(SIM_E_ARG, "scenario index %d out of range", s);
    if (!in) return h->fail(SIM_E_ARG, "in is NULL");
    if (step < 0) return h->fail(SIM_E_SHAPE, "step must be >= 0");
    if (h->calib()) return h->fail(SIM_E_STATE, "sim_set_state is not allowed in calibration mode");
    const fs::DevScen& J = h->job[s];
    int rc = h->hip(hipMemsetAsync(h->d_err(), 0, sizeof(int), h->st), "clear error flag");
    if (!rc) rc = h->hip(fs::launch_set_state(h->st, J, in, J.planes[h->parity], h->d_err()),
                         "set state");
    if (!rc) rc = refresh_worklist(h, true);
    if (!rc) rc = take_origin(h, step, false);
    int bad = 0;
    if (!rc) rc = h->hip(hipMemcpyAsync(&bad, h->d_err(), sizeof(int), hipMemcpyDeviceToHost,
                                        h->st), "read error flag");
    if (!rc) rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (rc) return rc;
    if (bad) return h->fail(SIM_E_ARG, "state has cells both burning and burned");
    h->step = step;
    return SIM_OK;
}

int sim_pignite(sim_handle* h, int32_t s, float* out) {
    if (!h) return SIM_E_ARG;
    if (s < 0 || s >= h->n) return h->fail(SIM_E_ARG, "scenario index %d out of range", s);
    if (!out) return h->fail(SIM_E_ARG, "out is NULL");
    return h->hip(fs::launch_pignite(h->st, h->d_jobs() + s, h->job[s], h->parity, out),
                  "pignite");
}

int sim_accumulator(sim_handle* h, int32_t s, float* out) {
    if (!h) return SIM_E_ARG;
    if (s < 0 || s >= h->n) return h->fail(SIM_E_ARG, "scenario index %d out of range", s);
    if (!out) return h->fail(SIM_E_ARG, "out is NULL");
    if (!h->calib()) return h->fail(SIM_E_STATE, "the accumulator needs SIM_F_CALIB");
    const fs::DevScen& J = h->job[s];
    return h->hip(hipMemcpyAsync(out, J.yhat, sizeof(float) * (size_t)J.H * J.W,
                                 hipMemcpyDeviceToDevice, h->st), "copy accumulator");
}

namespace {

// Adjoint job table for a run of T steps: one job per (scenario, segment).
int build_adjoint(sim_handle* h, int T) {
    const int nseg = (int)cdiv(T, h->ckpt_every);
    h->adj.clear();
    h->adj_tile_job.clear();
    int32_t g = 0;
    for (int i = 0; i < h->n; ++i) {
        const fs::DevScen& F = h->job[i];
        for (int sg = 0; sg < nseg; ++sg) {
            fs::DevScen J = F;
            const size_t idx = (size_t)i * h->L.nseg + sg;
            J.planes[0] = reinterpret_cast<uint32_t*>(h->ws + h->L.adj_planes[0][idx]);
            J.planes[1] = reinterpret_cast<uint32_t*>(h->ws + h->L.adj_planes[1][idx]);
            J.flags[0] = reinterpret_cast<uint8_t*>(h->ws + h->L.adj_flags[0][idx]);
            J.flags[1] = reinterpret_cast<uint8_t*>(h->ws + h->L.adj_flags[1][idx]);
            J.ckpt = F.ckpt + (int64_t)sg * 2 * h->L.s[i].PW;
            J.t_base = sg * h->ckpt_every;
            J.t_end = std::min((sg + 1) * h->ckpt_every, T);
            J.yhat = nullptr;
            J.tign = J.tout = nullptr;
            J.tile0 = g;
            const int32_t nt = J.tiles_r * J.tiles_c;
            h->adj_tile_job.insert(h->adj_tile_job.end(), nt, (int32_t)h->adj.size());
            g += nt;
            h->adj.push_back(J);
        }
    }
    int64_t off = 0;
    for (int i = 0; i < h->n; ++i) {
        for (int sg = 0; sg < nseg; ++sg) h->adj[(size_t)i * nseg + sg].lam_off = off;
        off += (int64_t)h->job[i].H * h->job[i].W;
    }
    h->adj_ntiles = g;
    int rc = h->hip(hipMemcpyAsync(h->ws + h->L.adj_jobs, h->adj.data(),
                                   sizeof(fs::DevScen) * h->adj.size(), hipMemcpyHostToDevice,
                                   h->st), "upload adjoint jobs");
    if (!rc) rc = h->hip(hipMemcpyAsync(h->ws + h->L.adj_tile_job, h->adj_tile_job.data(),
                                        sizeof(int32_t) * (size_t)g, hipMemcpyHostToDevice,
                                        h->st), "upload adjoint tiles");
    if (!rc) rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (!rc) h->adj_T = T;
    return rc;
}

int adjoint(sim_handle* h, const float* lam, double* grad) {
    if (h->stale)
        return h->fail(SIM_E_STATE, "the parameters changed after the run started; "
                       "sim_reset and sim_run again before the adjoint");
    const int T = h->step;
    if (T == 0)
        return h->hip(hipMemsetAsync(grad, 0, sizeof(double) * 4 * (size_t)h->n, h->st),
                      "zero gradient");
    fs::Rings rg = h->rings;
    rg.T = T;
    // both adjoints read the q8 table of the run's parameters
    if (int rc = ensure_qtable(h, T)) return rc;
    // gradient pass over every cell (per-block FP64 partials, then a fixed-order
    // reduction per scenario)
    auto gradient_pass = [&](bool from_maps) {
        auto* gp = reinterpret_cast<double*>(h->ws + h->L.gpart_tmap);
        const auto* bl0 = reinterpret_cast<const int32_t*>(h->ws + h->L.bl0);
        int r = h->hip(fs::launch_adjoint_cells(h->st, h->d_jobs(), bl0, h->n, h->L.tmap_blocks,
                                                lam, rg, gp, from_maps), "adjoint gradient");
        if (!r) r = h->hip(fs::launch_grad_reduce(h->st, gp, bl0, h->n, grad), "reduce gradient");
        return r;
    };
    if (h->adj_method == 1) return gradient_pass(true);
    // the segment jobs depend on T and the tiling only; parameters and seeds
    // come from the scenario jobs on the device, so a new gradient step of the
    // same length needs no host rebuild, upload or synchronisation
    int rc = SIM_OK;
    if (h->adj_T != T) rc = build_adjoint(h, T);
    if (rc) return rc;
    auto* d_adj = reinterpret_cast<fs::DevScen*>(h->ws + h->L.adj_jobs);
    auto* d_adj_tiles = reinterpret_cast<int32_t*>(h->ws + h->L.adj_tile_job);
    const int njobs = (int)h->adj.size();
    rc = h->hip(fs::launch_adj_params(h->st, d_adj, njobs, njobs / h->n, h->d_jobs()),
                "adjoint parameters");
    if (!rc) rc = h->hip(fs::launch_ckpt_load(h->st, d_adj, njobs, h->max_words), "load checkpoints");
    if (!rc) rc = h->hip(fs::launch_flags_init(h->st, d_adj, d_adj_tiles, h->adj_ntiles, 0,
                                               h->sh), "adjoint flags");
    auto* amask = reinterpret_cast<unsigned long long*>(h->ws + h->L.adj_masks);
    const int64_t anw = h->L.adj_mask_words;
    if (!rc && (h->ex.skip == 1 || h->ex.skip == 3))
        rc = h->hip(fs::launch_mask_init(h->st, d_adj, d_adj_tiles, h->adj_ntiles, 0, amask,
                                         h->L.adj_mask_words), "adjoint worklist");
    int alidx = 0;
    // the recompute records the burning slots of each cell it ignites at an
    // attached step; the gradient pass evaluates the cells with a record
    if (!rc) rc = h->hip(fs::launch_fill_u32(h->st, reinterpret_cast<uint32_t*>(h->ws + h->L.sm8),
                                             (size_t)cdiv(h->cell0.back(), 4), 0u),
                         "clear slot records");
    int parity = 0;
    unsigned long long* stats = nullptr;
    for (int off = 0; off < h->ckpt_every && !rc; ) {
        const int k = std::min(h->ex.depth, h->ckpt_every - off);
        fs::Sched sc{nullptr, nullptr, nullptr, h->L.adj_mask_words};
        if (h->ex.skip == 1 || h->ex.skip == 3) {
            sc.in = amask + anw * (alidx % 3);
            sc.out = amask + anw * ((alidx + 1) % 3);
            sc.clear = amask + anw * ((alidx + 2) % 3);
        }
        ++alidx;
        rc = h->hip(fs::launch_step(h->st, h->sh, true, d_adj, d_adj_tiles, h->adj_ntiles,
                                    parity, off, k, h->ex.skip, nullptr, rg, sc, h->grid_max,
                                    stats),
                    "adjoint recompute");
        parity ^= 1;
        off += k;
    }
    if (!rc) rc = gradient_pass(false);
    return rc;
}

}  // namespace

int sim_set_adjoint(sim_handle* h, int32_t method, int32_t r_first, int32_t r_between,
                    int32_t r_last) {
    if (!h) return SIM_E_ARG;
    if (method != SIM_ADJ_CHECKPOINT && method != SIM_ADJ_TIMEMAP)
        return h->fail(SIM_E_ARG, "unknown adjoint method %d", method);
    if (r_first >= 0 && (r_between < 0 || r_last < 0))
        return h->fail(SIM_E_ARG, "step-ring counts must be >= 0");
    h->adj_method = method;
    h->rings = fs::Rings{r_first < 0 ? -1 : r_first, r_first < 0 ? 0 : r_between,
                         r_first < 0 ? 0 : r_last, 0};
    return SIM_OK;
}

int sim_adjoint(sim_handle* h, const float* dL_dyhat, double* grad) {
    if (!h) return SIM_E_ARG;
    if (!dL_dyhat || !grad) return h->fail(SIM_E_ARG, "dL_dyhat and grad must be non-NULL");
    if (!h->calib()) return h->fail(SIM_E_STATE, "sim_adjoint needs SIM_F_CALIB");
    return adjoint(h, dL_dyhat, grad);
}

int sim_loss_grad(sim_handle* h, const uint8_t* target, int32_t kind, double* loss,
                  double* grad) {
    if (!h) return SIM_E_ARG;
    if (!target || !loss || !grad) return h->fail(SIM_E_ARG, "target, loss, grad must be non-NULL");
    if (kind < SIM_LOSS_BCE || kind > SIM_LOSS_MSE) return h->fail(SIM_E_ARG, "bad loss kind");
    if (!h->calib()) return h->fail(SIM_E_STATE, "sim_loss_grad needs SIM_F_CALIB");
    if (h->stale)
        return h->fail(SIM_E_STATE, "the parameters changed after the run started; "
                       "sim_reset and sim_run again before the loss and its gradient");
    float* lam = reinterpret_cast<float*>(h->ws + h->L.lam);
    int rc = h->hip(fs::launch_loss(h->st, h->d_jobs(),
                                    reinterpret_cast<const int64_t*>(h->ws + h->L.cell0), h->n,
                                    h->L.max_h, h->parity, target, kind, lam,
                                    reinterpret_cast<int*>(h->ws + h->L.box),
                                    reinterpret_cast<double*>(h->ws + h->L.part), loss),
                    "loss");
    if (rc) return rc;
    return adjoint(h, lam, grad);
}

int sim_set_wind(sim_handle* h, int32_t s, const float* wind_speed, const float* wind_dir_deg,
                 float wind_speed_scalar, float wind_dir_deg_scalar) {
    if (!h) return SIM_E_ARG;
    if (s < 0 || s >= h->n) return h->fail(SIM_E_ARG, "scenario index %d out of range", s);
    if (((uintptr_t)wind_speed | (uintptr_t)wind_dir_deg) & 3u)
        return h->fail(SIM_E_ARG, "wind fields must be 4-byte aligned");
    if (!wind_speed && (!std::isfinite(wind_speed_scalar) || wind_speed_scalar < 0.f))
        return h->fail(SIM_E_PARAM, "wind_speed_scalar must be finite, >= 0");
    if (!wind_dir_deg && !std::isfinite(wind_dir_deg_scalar))
        return h->fail(SIM_E_PARAM, "wind_dir_deg_scalar must be finite");
    if (h->calib() && h->step != 0)
        return h->fail(SIM_E_STATE, "in calibration mode the wind may change only at step 0");
    const fs::DevScen& J = h->job[s];
    int rc = h->hip(hipMemsetAsync(h->d_err(), 0, sizeof(int), h->st), "clear error flag");
    if (!rc) rc = h->hip(fs::launch_set_wind(h->st, J, wind_speed, wind_dir_deg, wind_speed_scalar,
                                             wind_dir_deg_scalar, const_cast<float4*>(J.rec),
                                             h->d_err()), "set wind");
    int bad = 0;
    if (!rc) rc = h->hip(hipMemcpyAsync(&bad, h->d_err(), sizeof(int), hipMemcpyDeviceToHost,
                                        h->st), "read error flag");
    if (!rc) rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (rc) return rc;
    h->q_dirty = h->q_params = true;
    h->d[s].f.wind_speed = wind_speed;
    h->d[s].f.wind_dir_deg = wind_dir_deg;
    h->d[s].f.wind_speed_scalar = wind_speed_scalar;
    h->d[s].f.wind_dir_deg_scalar = wind_dir_deg_scalar;
    if (bad) return h->fail(SIM_E_PARAM, "wind speed < 0 or non-finite wind (the record was "
                            "written; set a valid wind before running)");
    return SIM_OK;
}

int sim_ignite(sim_handle* h, int32_t s, const int32_t* cells, int32_t count) {
    if (!h) return SIM_E_ARG;
    if (s < 0 || s >= h->n) return h->fail(SIM_E_ARG, "scenario index %d out of range", s);
    if (count < 0) return h->fail(SIM_E_SHAPE, "count must be >= 0");
    if (count > 0 && !cells) return h->fail(SIM_E_ARG, "cells is NULL");
    if (h->calib()) return h->fail(SIM_E_STATE, "sim_ignite is not available in calibration mode");
    if (count == 0) return SIM_OK;
    int rc = h->hip(fs::launch_ignite(h->st, h->job[s], cells, count), "ignite");
    if (!rc) rc = refresh_worklist(h, false);   // both buffers were written
    if (!rc) rc = take_origin(h, h->step, false);
    return rc;
}

int sim_counts(sim_handle* h, int64_t* out) {
    if (!h) return SIM_E_ARG;
    if (!out) return h->fail(SIM_E_ARG, "out is NULL");
    return h->hip(fs::launch_counts(h->st, h->d_jobs(), h->n, h->parity, h->max_words,
                                    reinterpret_cast<long long*>(out)), "counts");
}

int sim_overlap(sim_handle* h, int32_t s, const uint8_t* target, int64_t* out) {
    if (!h) return SIM_E_ARG;
    if (s < 0 || s >= h->n) return h->fail(SIM_E_ARG, "scenario index %d out of range", s);
    if (!target || !out) return h->fail(SIM_E_ARG, "target and out must be non-NULL");
    return h->hip(fs::launch_overlap(h->st, h->job[s], h->parity, target,
                                     reinterpret_cast<long long*>(out)), "overlap");
}

int sim_metrics(sim_handle* h, const uint8_t* targets, int64_t* out) {
    if (!h) return SIM_E_ARG;
    if (!targets || !out) return h->fail(SIM_E_ARG, "targets and out must be non-NULL");
    if ((uintptr_t)out & 7u) return h->fail(SIM_E_ARG, "out must be 8-byte aligned");
    int64_t max_cells = 0;
    for (const auto& J : h->job) max_cells = std::max<int64_t>(max_cells, (int64_t)J.H * J.W);
    return h->hip(fs::launch_metrics(h->st, h->d_jobs(),
                                     reinterpret_cast<const int64_t*>(h->ws + h->L.cell0), h->n,
                                     h->parity, max_cells, targets,
                                     reinterpret_cast<long long*>(out)), "metrics");
}

int sim_arrival(sim_handle* h, int32_t s0, int32_t n, uint32_t* counts) {
    if (!h) return SIM_E_ARG;
    if (!counts || ((uintptr_t)counts & 3u)) return h->fail(SIM_E_ARG, "counts must be a 4-byte aligned device pointer");
    if (s0 < 0 || n < 1 || (int64_t)s0 + n > h->n)
        return h->fail(SIM_E_ARG, "scenario range [%d, %d) outside [0, %d)", s0, s0 + n, h->n);
    for (int s = s0 + 1; s < s0 + n; ++s)
        if (h->job[s].H != h->job[s0].H || h->job[s].W != h->job[s0].W)
            return h->fail(SIM_E_SHAPE, "scenario %d has a different grid shape than %d", s, s0);
    return h->hip(fs::launch_arrival(h->st, h->d_jobs(), h->job[s0], s0, n, h->parity, counts),
                  "arrival counts");
}

int sim_tielog(sim_handle* h, sim_tie* out, int64_t capacity, int64_t* count) {
    static_assert(sizeof(sim_tie) == sizeof(fs::TieRec), "tie record layout");
    static_assert(SIM_TIELOG_CAP == fs::kTieLogCap, "tie log capacity");
    if (!h) return SIM_E_ARG;
    if (!(h->flags & SIM_F_TIELOG)) return h->fail(SIM_E_STATE, "the handle has no tie log (SIM_F_TIELOG)");
    if (!count || capacity < 0 || (capacity > 0 && !out))
        return h->fail(SIM_E_ARG, "count must be non-NULL and out non-NULL when capacity > 0");
    unsigned long long n = 0;
    int rc = h->hip(hipMemcpyAsync(&n, h->ws + h->L.tie_n, sizeof n, hipMemcpyDeviceToHost, h->st),
                    "read tie count");
    if (!rc) rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (rc) return rc;
    const int64_t m = std::min<int64_t>(std::min<int64_t>((int64_t)n, capacity), SIM_TIELOG_CAP);
    if (m > 0)
        rc = h->hip(hipMemcpyAsync(out, h->ws + h->L.tielog, sizeof(sim_tie) * (size_t)m,
                                   hipMemcpyDeviceToDevice, h->st), "copy tie log");
    if (!rc) rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (!rc) *count = (int64_t)n;
    return rc;
}

int sim_stats(sim_handle* h, uint64_t out[4]) {
    if (!h || !out) return SIM_E_ARG;
    unsigned long long v[4] = {0, 0, 0, 0};
    int rc = h->hip(hipMemcpyAsync(v, h->d_stats(), sizeof v, hipMemcpyDeviceToHost, h->st),
                    "read stats");
    if (!rc) rc = h->hip(hipStreamSynchronize(h->st), "synchronise");
    if (rc) return rc;
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
    out[3] = h->launches;
    return SIM_OK;
}

const char* sim_last_error(const sim_handle* h) {
    return h ? h->err.c_str() : g_init_error.c_str();
}

void sim_destroy(sim_handle* h) {
    if (!h) return;
    if (h->static_dev >= 0) {
        // the next static handle on this device reuses the array: let this
        // handle's queued work finish before the array is handed out again
        (void)hipStreamSynchronize(h->st);
        release_static(h);
    }
    delete h;
}

}  // extern "C"
