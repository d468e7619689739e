// internal.h -- device-side descriptors and kernel launchers of libfiresim.
//
// Data layout in HBM (per scenario, all inside the caller's workspace):
//   rec     float4 per cell: (F, V, V cos(theta_w), V sin(theta_w)) with
//           F = (1 + p_veg)(1 + p_den), the fuel factors of Eq. 2 multiplied
//           once, and the wind heading resolved into east/north components.
//   th8     8 floats per cell: the Eq. 1 slope angle (degrees) from each
//           neighbour slot toward the cell (static, built once).
//   q8      8 floats per cell: f_p(p_propagate) of the edge from each
//           neighbour slot into the cell for the current parameters (Eq. 2-5),
//           rebuilt at the start of a run whenever parameters or the run
//           changed.  Slot order: (dr, dc) row by row, centre skipped.
//   fuel    one bit per cell (F > 0), rows of `pitch` 32-bit words.
//   planes  two ping-pong buffers; each holds the burning bit-plane followed
//           by the burned bit-plane (2 * H * pitch words): 2 bits per cell.
//   flags   per tile and per buffer parity: bit 0 = some cell of the tile is
//           burning, bit 1 = both ping-pong buffers hold the same tile.
//   yhat    FP32 accumulator (calibration), ckpt state checkpoints.
// Bit b of word w in row r is the cell (r, 32 w + b).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fs {

struct DevScen {
    int32_t H, W, pitch;       // pitch: 32-bit words per row
    int32_t tiles_r, tiles_c;  // tile grid of the current execution shape
    int32_t tile0;             // first global tile index of this job
    int32_t t_base;            // step index offset of this job
    int32_t t_end;             // last step this job may produce
    uint32_t scen_id;
    uint32_t seed_lo, seed_hi;
    float inv_l, inv_l_diag;   // 1 / l and 1 / (sqrt(2) l) of Eq. 1
    float p_h, a, c1, c2, p_continue, c;
    int32_t sidx;              // index of the scenario in its handle
    const float* elev;         // caller's elevation field
    const float4* rec;         // per-cell record
    const float* th8;          // slope (Eq. 1, degrees) toward each of the 8 neighbours
    float* q8;                 // f_p(p_propagate) of each of the 8 incoming edges (per run)
    const uint32_t* init;      // initial burning bit-plane (H * pitch words, packed at set-up)
    const uint32_t* fuel;      // fuel bit-plane
    uint32_t* planes[2];       // ping-pong state buffers
    uint8_t* flags[2];         // per-tile flags, per parity
    float* yhat;               // accumulator or nullptr
    int32_t* tign;             // step each cell ignited (0: initially burning) or nullptr
    int32_t* tout;             // step each cell burnt out, or nullptr
    uint32_t* ckpt;            // checkpoint store (forward) / own segment (adjoint)
    uint8_t* sm8;              // burning slots of each cell that ignited at an attached
                               // step, recorded by the checkpoint adjoint's recompute
                               // (0: none); nullptr outside calibration
    int64_t lam_off;           // offset of this scenario's dL/dyhat grid
    // Blocks of 32 x 32 cells (block (br, bc): rows 32 br .. 32 br + 31, word
    // bc of each row), one bit each, rows of cdiv(pitch, 32) words: blocks
    // with a burning cell at the propagation table's origin step, the same
    // grown along the rows, and grown along the columns too (the blocks the
    // table covers)
    uint32_t* qburn;
    uint32_t* qrow;
    uint32_t* qneed;
    void* tielog;              // near-tie records (sim_tie layout) or nullptr
    unsigned long long* tie_n; // number of trials logged
};

// Near-tie log: capacity and window of the records (|u - p| <= kTieLogEps).
constexpr long long kTieLogCap = 1 << 20;
constexpr float kTieLogEps = 2e-5f;
struct TieRec {
    int32_t scenario, step;
    int64_t cell;
    float p, u;
    int32_t ignited, reserved;
};

// Step-ring attach set of the adjoint (Sec. 2.3): ignition steps t with
// t <= first, or t > T - last, or t one of `between` steps spread evenly in
// between; first < 0 attaches every step.
struct Rings {
    int32_t first, between, last, T;
};

// Worklist of a launch: bit g of `in` marks global tile g for processing;
// processed tiles that still hold fire (or changed) mark themselves and their
// 8 neighbour tiles in `out` for the next launch; `clear` (the mask of the
// launch after next) is zeroed.  in == nullptr: every tile is launched.
struct Sched {
    const unsigned long long* in;
    unsigned long long* out;
    unsigned long long* clear;
    int32_t nwords;
};

struct TileShape {
    int tr, tc, km;            // rows, words, halo depth (max steps per launch)
    int nt;                    // work-group size; 0 = the shape's default (first entry)
};

// Kernel launchers (kernels.hip).  All enqueue on `st` and return the launch
// status; they assume arguments were validated by the caller.
hipError_t launch_prologue(hipStream_t st, const DevScen* d_job, const DevScen& job,
                           const float* p_veg, const float* p_den, const float* ws,
                           const float* wd, float ws0, float wd0, const uint8_t* ign,
                           float4* rec, uint32_t* fuel, float* yhat, int* d_err);
// Slope table th8 of one scenario from its elevation (after the prologue),
// or from the paper-layout H x W x 3 x 3 slope tensor when slope9 != nullptr
// (non-finite entries set bit 64 of *d_err).
hipError_t launch_slopes(hipStream_t st, const DevScen& job, float* th8, const float* slope9,
                         int* d_err);
// Wind of one scenario: rewrite (V, V cos, V sin) of rec (F kept).
hipError_t launch_set_wind(hipStream_t st, const DevScen& job, const float* ws, const float* wd,
                           float ws0, float wd0, float4* rec, int* d_err);
// Set listed cells burning in both ping-pong buffers (spotting).
hipError_t launch_ignite(hipStream_t st, const DevScen& job, const int32_t* cells, int32_t count);
// out[2s], out[2s+1] += burning / burned counts of every job (out zeroed first).
hipError_t launch_counts(hipStream_t st, const DevScen* d_jobs, int32_t n, int32_t parity,
                         int64_t max_words, long long* out);
// out[4 s ..] = (|A & B|, |A | B|, |A|, |B|) of every job s: A its affected
// cells, B the non-zero cells of its target grid (concatenated at d_cell0[s]).
hipError_t launch_metrics(hipStream_t st, const DevScen* d_jobs, const int64_t* d_cell0, int32_t n,
                          int32_t parity, int64_t max_cells, const uint8_t* target,
                          long long* out);
// counts[j] += scenarios s0 .. s0+n-1 (shape of J0 = job s0) in which j is affected
hipError_t launch_arrival(hipStream_t st, const DevScen* d_jobs, const DevScen& J0, int32_t s0,
                          int32_t n, int32_t parity, uint32_t* counts);
// out = (|A & B|, |A | B|) for affected cells A of one job and target B.
hipError_t launch_overlap(hipStream_t st, const DevScen& job, int32_t parity, const uint8_t* target,
                          long long* out);
// box[s] = (r0, r1, c0, c1), the bounding box of the burning cells of every
// scenario in planes[parity] (r1 < r0: nothing burns), and the qburn bits of
// the 32 x 32 blocks holding a burning cell; qburn_all (qwords words) is the
// bit array of all scenarios, cleared first.
hipError_t launch_bbox(hipStream_t st, const DevScen* d_jobs, int32_t n, int32_t parity,
                       int64_t max_words, int4* box, uint32_t* qburn_all, int64_t qwords);
// Largest reach (in blocks of 32 cells) for which the table is restricted to
// the blocks near a burning block (qneed); beyond it the box alone bounds it.
constexpr int kMaxBlockReach = 16;
// Propagation table q8 of every scenario for the current parameters, over the
// cells within `reach` of box[s] (the only cells that can have an ignition
// trial in the next `reach` steps) and, when ceil(reach / 32) <=
// kMaxBlockReach, in the blocks within ceil(reach / 32) blocks of a qburn
// block; qbox (n) and cell0q (n + 1) are scratch for the regions and their
// prefix sums; max_cells bounds their total, max_qwords the bit words of a
// scenario.
hipError_t launch_qtable(hipStream_t st, const DevScen* d_jobs, const int4* box, int32_t n,
                         int32_t reach, int64_t max_cells, int64_t max_qwords, int4* qbox,
                         int64_t* cell0q);
// State of every scenario back to its initial burning cells (both ping-pong
// buffers; with maps, also the accumulator and time maps); d_ib0 = n + 1
// prefix sums of the blocks per scenario, ceil(H * pitch / 256).
hipError_t launch_init_state(hipStream_t st, const DevScen* d_jobs, const int32_t* d_ib0,
                             int32_t n, int32_t nblocks, const int64_t* d_cell0,
                             int64_t total_cells, bool maps);
// Time-map adjoint: one pass over every cell of every scenario; bl0 = n + 1
// prefix sums of ceil(cells / 256) per scenario; writes gpart[block][4].
// Gradient pass of the adjoints: per-block FP64 partials of
// lambda_j * d p_ignite_j / d theta over the cells that ignited at attached
// steps, their burning slots from the ignition / burn-out maps (from_maps,
// time-map adjoint) or from the slot masks the recompute recorded (sm8).
hipError_t launch_adjoint_cells(hipStream_t st, const DevScen* d_jobs, const int32_t* d_bl0,
                                int32_t n, int32_t nblocks, const float* lam, Rings rings,
                                double* gpart, bool from_maps);
hipError_t launch_set_state(hipStream_t st, const DevScen& job, const uint8_t* in,
                            uint32_t* planes, int* d_err);
hipError_t launch_get_state(hipStream_t st, const DevScen& job, const uint32_t* planes,
                            uint8_t* out);
hipError_t launch_flags_init(hipStream_t st, const DevScen* d_jobs, const int32_t* d_tile_job,
                             int32_t ntiles, int32_t parity, TileShape sh);
bool step_shape_supported(TileShape sh, bool adj);
// The compiled forward shapes (at most `max`); returns how many.
int step_shapes(TileShape* out, int max);
hipError_t launch_step(hipStream_t st, TileShape sh, bool adj, const DevScen* d_jobs,
                       const int32_t* d_tile_job, int32_t ntiles, int32_t parity,
                       int32_t t_off, int32_t ksteps, int32_t skip, const float* lam,
                       Rings rings, Sched sched, int32_t grid, unsigned long long* d_stats);
// Worklist for the first launch after a state change: every tile whose 3 x 3
// tile neighbourhood holds a burning cell (from the flags of `parity`); the
// three masks (3 * nwords words) are cleared first.
hipError_t launch_mask_init(hipStream_t st, const DevScen* d_jobs, const int32_t* d_tile_job,
                            int32_t ntiles, int32_t parity, unsigned long long* masks,
                            int32_t nwords);
// Copy every job's planes[parity] into the other buffer (both ping-pong
// buffers equal, so tiles left out of a worklist stay consistent).
hipError_t launch_dup_planes(hipStream_t st, const DevScen* d_jobs, int32_t n, int32_t parity,
                             int64_t max_words);
// Copy each job's current planes into checkpoint slot `slot` (forward jobs).
hipError_t launch_ckpt_save(hipStream_t st, const DevScen* d_jobs, int32_t n, int32_t parity,
                            int32_t slot, int64_t max_words);
// Copy each adjoint job's checkpoint into its planes[0].
hipError_t launch_ckpt_load(hipStream_t st, const DevScen* d_jobs, int32_t n, int64_t max_words);
struct ParamBlock {
    int32_t first, count;
    float v[64][5];
};
hipError_t launch_set_params(hipStream_t st, DevScen* d_jobs, const ParamBlock& pb);
struct SeedBlock {
    int32_t first, count;
    uint32_t lo[64], hi[64];
};
hipError_t launch_set_seeds(hipStream_t st, DevScen* d_jobs, const SeedBlock& sb);
// theta: device, n rows of (p_h, a, c1, c2) for the n jobs; rows that are not
// finite or have p_h < 0 keep the job's parameters and add 1 to *rejected.
hipError_t launch_set_theta(hipStream_t st, DevScen* d_jobs, int32_t n, const float* theta,
                            int* rejected);
// The checkpoint adjoint's per-segment jobs (nseg per scenario, scenario-major)
// take the current parameters and Philox keys of their scenario's job.
hipError_t launch_adj_params(hipStream_t st, DevScen* d_adj, int32_t nadj, int32_t nseg,
                             const DevScen* d_jobs);
hipError_t launch_pignite(hipStream_t st, const DevScen* d_job, const DevScen& job,
                          int32_t parity, float* out);
// Eq. 10 for each of the n scenarios (accumulators from their descriptors;
// y and lambda concatenated, scenario i at d_cell0[i]): writes lambda =
// dL/dyhat and loss_out[i].  The crop box comes from the state in
// planes[parity] (calibration handles: the accumulator is non-zero exactly on
// the cells that burn or burned) and the target.  d_box holds 4 n ints,
// d_part 2 n ceil(max_h / 4) doubles.
hipError_t launch_loss(hipStream_t st, const DevScen* d_jobs, const int64_t* d_cell0, int32_t n,
                       int32_t max_h, int32_t parity, const uint8_t* y, int32_t kind,
                       float* lambda, int* d_box, double* d_part, double* loss_out);
// grad[s] = sum of gpart[g] over blocks g in [ranges[s], ranges[s+1]).
hipError_t launch_grad_reduce(hipStream_t st, const double* gpart, const int32_t* d_ranges,
                              int32_t n, double* grad);
hipError_t launch_fill_u32(hipStream_t st, uint32_t* p, size_t n, uint32_t v);

}  // namespace fs
