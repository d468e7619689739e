/*
 * firesim.h -- C ABI of the MI355X (gfx950) wildfire cellular-automaton library.
 *
 * The library advances the stochastic cellular automaton of "PyTorchFire: A
 * GPU-Accelerated Wildfire Simulator with Differentiable Cellular Automata"
 * (Xia & Cheng, Environmental Modelling & Software 188, 2025) on the GPU:
 *   - inputs, parameters and outputs as listed in Sec. 2.1;
 *   - per-edge propagation probability, Eq. 1-5 (slope from elevation, wind,
 *     fuel, f_p(x) = tanh(c x) with c = 1.1486328125 rounded to FP32);
 *   - ignition probability over the Moore neighbourhood, Eq. 9;
 *   - the transition rules of Sec. 2.2 (burnable -> burning w.p. p_ignite when
 *     a neighbour burns, burning stays burning w.p. p_continue, burned is
 *     absorbing), all decided from the state at t-1;
 *   - the accumulator of p_ignite at the ignition step (Sec. 2.2, data flow)
 *     and the gradient of the Eq. 10 loss through it (Sec. 2.3).
 *
 * Conventions shared by every call
 *   - Grids are row-major H x W, row 0 = north, columns run east.  Wind
 *     direction is the heading the wind blows toward, degrees counter-
 *     clockwise from east.  Cells outside the grid never burn.
 *   - Random numbers: Philox4x32-10 with key = seed and counter
 *     (cell, 0, step, scenario_id), cell = r*W + c, step = index of the state
 *     being produced (1 for the first step).  Word 0 gives the ignition draw,
 *     word 1 the continue draw, each (w >> 8) * 2^-24.  A cell ignites iff
 *     draw < p_ignite (FP32); it keeps burning iff draw < p_continue.
 *   - Ownership: every pointer in sim_fields, every output buffer and the
 *     workspace are DEVICE pointers owned by the caller.  They must stay valid
 *     until sim_destroy.  The library never allocates device memory.
 *   - Streams: all work is enqueued on the stream given to sim_init; calls
 *     return once the work is enqueued (sim_init also waits for its
 *     validation result).  Results are valid after the stream synchronises.
 *   - Errors: every int-returning call returns SIM_OK (0) or a negative
 *     SIM_E_* code and records a message readable with sim_last_error.
 *     Argument checks run before any GPU work, so a rejected call has no
 *     effect.  No C++ exception crosses this boundary.
 *   - Thread safety: a handle must not be used from two threads at once.
 */
#ifndef FIRESIM_H
#define FIRESIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Exported entry points (the library is built with hidden visibility). */
#if defined(__GNUC__) || defined(__clang__)
#define SIM_API __attribute__((visibility("default")))
#else
#define SIM_API
#endif

#define SIM_OK 0
#define SIM_E_ARG (-1)        /* null / misaligned pointer, bad enum value   */
#define SIM_E_SHAPE (-2)      /* H, W, n, T, tile or depth out of range      */
#define SIM_E_PARAM (-3)      /* non-finite or out-of-range parameter/field  */
#define SIM_E_WORKSPACE (-4)  /* workspace too small or misaligned           */
#define SIM_E_HIP (-5)        /* a HIP runtime call failed                   */
#define SIM_E_STATE (-6)      /* call not valid in the handle's state        */

/* sim_init flags */
#define SIM_F_CALIB 1u        /* keep the accumulator and state checkpoints   */
#define SIM_F_STATS 2u        /* count processed tiles, trials and near ties  */
#define SIM_F_TIELOG 4u       /* log ignition trials with |draw - p| <= 2e-5   */

/* Near-tie log (SIM_F_TIELOG): one record per ignition trial whose uniform
 * draw lies within 2e-5 of its FP32 p_ignite (Eq. 9), at most SIM_TIELOG_CAP
 * records since the last reset.  Such trials are the ones whose decision may
 * differ from an FP64 evaluation of the same step. */
#define SIM_TIELOG_CAP (1 << 20)
typedef struct {
    int32_t scenario;   /* index of the scenario in the handle */
    int32_t step;       /* step t of the trial (S(t) is being produced) */
    int64_t cell;       /* r * W + c */
    float p_ignite;     /* FP32 p_ignite of the trial */
    float draw;         /* the uniform draw u of the trial */
    int32_t ignited;    /* u < p_ignite */
    int32_t reserved;
} sim_tie;

/* loss kinds of sim_loss_grad (Eq. 10) */
#define SIM_LOSS_BCE 0        /* BCE-with-logits over the bounding-box crop   */
#define SIM_LOSS_BCE_MSE 1    /* BCE + MSE of 4x4, stride-4 average pools     */
#define SIM_LOSS_MSE 2        /* MSE term only                                */

typedef struct sim_handle sim_handle;

/* The five parameters of Sec. 2.1 (p_continue is never differentiated). */
typedef struct {
    float p_h, a, c1, c2, p_continue;
} sim_params;

/* Input fields of one scenario (Sec. 2.1).  Device pointers, FP32, H*W,
 * row-major, caller-owned.  p_veg = -1 (or p_den = -1) marks a cell without
 * fuel (Sec. 2.2: a small enough p_veg gives zero propagation); values below
 * -1 are rejected.  Slope is derived from the elevation with Eq. 1 in place of
 * the paper's H x W x 3 x 3 slope tensor unless slope_deg is given.
 * wind_speed / wind_dir_deg may be NULL, in which case the two scalars apply
 * to every cell. */
typedef struct {
    const float* p_veg;
    const float* p_den;
    const float* elevation_m;
    const float* wind_speed;
    const float* wind_dir_deg;
    float wind_speed_scalar;
    float wind_dir_deg_scalar;
    const uint8_t* init_burning;   /* H*W bytes, non-zero = burning at t = 0 */
    /* Optional: the paper's slope tensor (Sec. 2.1), H*W*3*3 FP32 degrees;
     * element [r][c][dr+1][dc+1] is theta_s of Eq. 4 for the edge from
     * neighbour (r+dr, c+dc) into (r, c), positive when the spread runs
     * uphill.  When non-NULL it replaces Eq. 1 and elevation_m may be NULL. */
    const float* slope_deg;
} sim_fields;

/* One scenario.  cell_m is l of Eq. 1 in metres; seed keys the Philox stream;
 * scenario_id is the fourth counter word (distinct ids give independent
 * streams under one seed). */
typedef struct {
    int32_t H, W;
    float cell_m;
    uint32_t scenario_id;
    uint64_t seed;
    sim_params params;
    sim_fields f;
} sim_desc;

/* Execution shape: rows x words of one tile (a word is 32 cells), steps per
 * launch (temporal block depth, 1 <= depth <= tile_rows and <= 32), and how
 * tiles with no burning cell within reach are skipped: 0 = every tile is
 * processed, 1 = a device-built worklist (tiles that burn mark their
 * neighbours for the next launch; a grid of resident work-groups walks it),
 * 2 = every tile is launched and tests its neighbours' flags, 3 = every tile
 * is launched and tests its bit of the worklist (one read; mode 1's lists,
 * mode 2's launch shape and register budget).  threads is the
 * work-group size (0 = the shape's default: 256 lanes for tiles of up to 16
 * rows, 512 for 32-row tiles, which are also compiled with 256).  Every shape
 * produces bit-identical states. */
typedef struct {
    int32_t tile_rows, tile_words, depth, skip, threads;
} sim_exec;

/* Bytes of workspace sim_init needs for these scenarios.  ckpt_every and
 * T_max size the checkpoint store and are only used with SIM_F_CALIB.
 * Returns 0 when the arguments are invalid. */
SIM_API size_t sim_workspace_size(const sim_desc* descs, int32_t n, uint32_t flags,
                          int32_t ckpt_every, int32_t T_max);

/* Create a handle over n scenarios.  `descs` is a host array of n entries.
 * Validates every field on the device (p_veg, p_den >= -1, finite elevation,
 * wind >= 0 and finite), builds the per-cell records and the fuel bit-plane,
 * sets the state to init_burning at step 0, and synchronises `stream` once to
 * read the validation result.  `workspace` must be 256-byte aligned and at
 * least sim_workspace_size(...) bytes.  `stream` is a hipStream_t (NULL = the
 * default stream).  On failure *out is NULL and sim_last_error(NULL) says why. */
SIM_API int sim_init(sim_handle** out, const sim_desc* descs, int32_t n, void* workspace,
             size_t ws_bytes, void* stream, uint32_t flags, int32_t ckpt_every,
             int32_t T_max);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): sim_init without a
 * workspace argument.  The handle's workspace is a 128 MiB array in the
 * library's static device memory, one copy per GPU, which that GPU holds
 * from the first call on it until the process ends.  The call allocates
 * nothing on the device (no hipMalloc, no allocating library routine); the
 * caller still owns the fields and every output buffer.
 *   - Size: scenarios whose sim_workspace_size exceeds
 *     SIM_STATIC_SCRATCH_BYTES are rejected with SIM_E_WORKSPACE (nothing is
 *     enqueued).  One scenario fits up to about 1280 x 1280 cells (forward)
 *     or 1120 x 1120 (calibration, 200 steps, checkpoints every 20).
 *   - One static handle per GPU at a time: the array is the handle's whole
 *     workspace, so while one exists on the current device another
 *     sim_init_static there returns SIM_E_STATE.  sim_destroy of a static
 *     handle waits for its stream, then releases the array.
 *   - The array keeps what the last handle left in it; set-up initialises
 *     every part the kernels read, exactly as sim_init does for a reused
 *     workspace.  Work enqueued by a destroyed handle's caller on other
 *     streams after sim_destroy must not touch the array.
 *   - The device is the current HIP device at the call; `stream` must belong
 *     to it.  Arguments, flags, errors and the behaviour of every other call
 *     on the handle are those of sim_init. */
#define SIM_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
SIM_API int sim_init_static(sim_handle** out, const sim_desc* descs, int32_t n, void* stream,
                            uint32_t flags, int32_t ckpt_every, int32_t T_max);

/* Choose the execution shape (default: 32 rows x 2 words, depth 32, worklist skipping;
 * sim_autotune picks one by timing).  Only whitelisted shapes are compiled; others give
 * SIM_E_SHAPE. */
SIM_API int sim_set_exec(sim_handle* h, const sim_exec* e);
SIM_API int sim_get_exec(const sim_handle* h, sim_exec* e);

/* Build the per-edge propagation table (Eq. 2-5 for every edge the fire can
 * reach in the next T steps) now.  sim_run builds it itself when needed
 * (after sim_set_params, sim_set_wind, sim_set_state, sim_ignite, after
 * sim_reset unless the table was last built around the reset state under the
 * current parameters and wind, or when a run goes past the steps it was built
 * for); calling sim_prepare
 * first keeps that work out of a timed region or a captured launch sequence.
 * The table covers the cells within (step + T - origin) cells of the burning
 * cells at the origin step (the last reset, set_state or ignite). */
SIM_API int sim_prepare(sim_handle* h, int32_t T);

/* Autotuner: times every compiled execution shape (skipping on; temporal
 * depth: T_probe steps in as few launches as the shape's halo allows, spread
 * evenly, e.g. 10 for 20 steps on a 16-step halo) over T_probe steps from the
 * current state, keeps the fastest and writes it to *best (nullable).  The state and step counter
 * are restored afterwards, so results do not depend on having tuned.  Waits
 * for the stream.  Not available in calibration mode (SIM_E_STATE). */
SIM_API int sim_autotune(sim_handle* h, int32_t T_probe, sim_exec* best);

/* Replay each distinct launch sequence of sim_run (same start step, parity,
 * T and shape) as one captured HIP graph (on by default; 0 turns it off and
 * frees the captured graphs).  Falls back to direct launches if capture is
 * not possible. */
SIM_API int sim_use_graphs(sim_handle* h, int32_t on);

/* Advance every scenario by T >= 0 steps (Sec. 2.2 transition rules).  In
 * calibration mode the accumulator records p_ignite at each ignition and the
 * state is checkpointed every ckpt_every steps; the run may not go past
 * T_max steps from the last reset. */
SIM_API int sim_run(sim_handle* h, int32_t T);
SIM_API int sim_step(sim_handle* h);

/* Steps taken since the last reset (host-side counter). */
SIM_API int sim_get_step(const sim_handle* h, int32_t* step);

/* Replace the parameters: `per_scenario` is a host array of n entries.
 * Takes effect from the next step.  In calibration mode, a change after the
 * run has started (step != 0) leaves the run's checkpoints and time maps
 * under the old parameters: sim_adjoint and sim_loss_grad then return
 * SIM_E_STATE until the next sim_reset. */
SIM_API int sim_set_params(sim_handle* h, const sim_params* per_scenario);

/* The calibrated parameters theta = (p_h, a, c1, c2) of Algorithm 1 from
 * device memory, for a calibration loop whose optimiser step runs on the GPU
 * (no host round trip between gradient steps).  `theta`: device pointer,
 * 4-byte aligned, n rows of 4 float32, read on the handle's stream in stream
 * order (the caller orders its writes before the call, e.g. on the same
 * stream).  p_continue is kept.  Rows are checked on the device: a row with a
 * non-finite value or p_h < 0 leaves that scenario's parameters unchanged
 * and is counted; sim_params_rejected returns the count.  Otherwise as
 * sim_set_params (the propagation table is rebuilt, and in calibration mode a
 * change after step 0 makes the adjoint wait for the next sim_reset). */
SIM_API int sim_set_params_device(sim_handle* h, const float* theta);

/* Number of parameter rows sim_set_params_device rejected since the handle
 * was made or the last call of this function (which clears it); waits for
 * the handle's stream. */
SIM_API int sim_params_rejected(sim_handle* h, int32_t* count);

/* Restore every scenario to init_burning at step 0 and clear the
 * accumulator (Algorithm 1, model.reset).  `seeds` (host, n entries) replaces
 * the Philox keys, or is NULL to keep them.  A propagation table built around
 * the reset state under the current parameters and wind stays valid (it does
 * not depend on the seeds), so runs of an ensemble that only changes seeds
 * do not rebuild it. */
SIM_API int sim_reset(sim_handle* h, const uint64_t* seeds);

/* Copy scenario s's state into `out` (device, 2*H*W bytes: channel 0 =
 * burning, channel 1 = burned, Sec. 2.1 output), or set it from `in` (same
 * layout, channels must not both be set) and declare it to be the state after
 * `step` steps.  sim_set_state is not allowed in calibration mode. */
SIM_API int sim_get_state(sim_handle* h, int32_t s, uint8_t* out);
SIM_API int sim_set_state(sim_handle* h, int32_t s, const uint8_t* in, int32_t step);

/* Ignition-probability map of Eq. 9 for scenario s's current state
 * (the paper's "internal function"): device FP32 H*W; 0 for cells that are
 * not burnable or have no burning neighbour. */
SIM_API int sim_pignite(sim_handle* h, int32_t s, float* out);

/* Accumulator of scenario s (calibration mode): p_ignite at the step each
 * cell ignited, 1 for initially burning cells, 0 otherwise.  Device FP32 H*W. */
SIM_API int sim_accumulator(sim_handle* h, int32_t s, float* out);

/* Gradient of sum_s sum_j dL_dyhat[s][j] * yhat[s][j] with respect to
 * (p_h, a, c1, c2) for each scenario, with states held constant (Sec. 2.3:
 * only p_ignite of ignited cells carries gradient).  Recomputes every
 * checkpoint segment of the last run.  dL_dyhat: device FP32, the n grids
 * concatenated; grad: device FP64, n x 4.  Calibration mode only. */
SIM_API int sim_adjoint(sim_handle* h, const float* dL_dyhat, double* grad);

/* Adjoint used by sim_adjoint and sim_loss_grad.
 *   SIM_ADJ_CHECKPOINT (default): recompute every checkpoint segment of the
 *     last run (all segments of all scenarios in one launch sequence),
 *     recording the burning neighbours at t_j - 1 of every cell j it ignites.
 *   SIM_ADJ_TIMEMAP: no recompute; the forward records each cell's ignition
 *     and burn-out steps, from which those neighbours are rebuilt exactly.
 * Both then evaluate the same per-cell terms in one pass over the cells,
 * summed in the same fixed order.
 * Step rings (Sec. 2.3, "update by step rings"): only cells ignited at an
 * attached step contribute -- steps 1..r_first, the last r_last steps, and
 * r_between steps spread evenly in between (step r_first + round(k * span /
 * (r_between + 1)), k = 1..r_between, span = T - r_first - r_last).
 * r_first < 0 attaches every step (the default). */
#define SIM_ADJ_CHECKPOINT 0
#define SIM_ADJ_TIMEMAP 1
SIM_API int sim_set_adjoint(sim_handle* h, int32_t method, int32_t r_first, int32_t r_between,
                            int32_t r_last);

/* Eq. 10 loss of the accumulator against `target` (device uint8, the n grids
 * concatenated, non-zero = observed fire) and its gradient: loss is device
 * FP64 n, grad device FP64 n x 4 (p_h, a, c1, c2).  Calibration mode only. */
SIM_API int sim_loss_grad(sim_handle* h, const uint8_t* target, int32_t loss_kind, double* loss,
                  double* grad);

/* Replace scenario s's wind (Algorithm 1 updates the wind per observation):
 * device FP32 H*W fields or NULL for the scalars, as in sim_fields.  Takes
 * effect from the next step.  In calibration mode only at step 0 (right
 * after sim_reset), so that a run and its adjoint see one wind.  Validates on
 * the device and waits for the stream; the fields are read during the call
 * only (unlike sim_fields, they need not outlive it). */
SIM_API int sim_set_wind(sim_handle* h, int32_t s, const float* wind_speed,
                         const float* wind_dir_deg, float wind_speed_scalar,
                         float wind_dir_deg_scalar);

/* Spotting (Sec. 2.2): set `count` cells of scenario s burning in place, as
 * extra ignition points, before the next step.  `cells` is a device int32
 * array of r*W + c indices; indices outside the grid and cells already
 * burned are ignored.  Not available in calibration mode. */
SIM_API int sim_ignite(sim_handle* h, int32_t s, const int32_t* cells, int32_t count);

/* Burning and burned cell counts of every scenario (device int64, n x 2):
 * the affected-cell counts of Eq. 12. */
SIM_API int sim_counts(sim_handle* h, int64_t* out);

/* Overlap of scenario s's affected cells (burning or burned) with `target`
 * (device uint8 H*W, non-zero = affected): out (device int64 x 2) =
 * (|A intersect B|, |A union B|); Eq. 11's Jaccard index is their ratio. */
SIM_API int sim_overlap(sim_handle* h, int32_t s, const uint8_t* target, int64_t* out);

/* Eq. 11 and Eq. 12 against observed maps, all scenarios in one launch:
 * `targets` is device uint8, the n grids concatenated (non-zero = observed
 * affected cell); out (device int64, n x 4) receives per scenario
 * (|A intersect B|, |A union B|, |A|, |B|), A = the scenario's affected cells
 * (burning or burned) at the current step, B = its target's.  Jaccard (Eq. 11)
 * is the first over the second; Eq. 12 sums |A| - |B| in absolute value over
 * the observation times. */
SIM_API int sim_metrics(sim_handle* h, const uint8_t* targets, int64_t* out);

/* Probability of arrival from an ensemble of runs (Sec. 1): counts[j] (device
 * uint32 H*W, zeroed by the caller) += the number of scenarios s0 .. s0+n-1
 * in which cell j is affected (burning or burned).  The n scenarios must share
 * one grid shape (SIM_E_SHAPE otherwise); typically they differ only in seed.
 * counts / (number of runs accumulated) is the arrival-probability map. */
SIM_API int sim_arrival(sim_handle* h, int32_t s0, int32_t n, uint32_t* counts);

/* Copy the near-tie log (handle created with SIM_F_TIELOG) to `out` (device
 * array of `capacity` records, nullable when capacity is 0): the first
 * min(logged, capacity, SIM_TIELOG_CAP) records, in no particular order.
 * *count (host) receives the number of trials logged since the last reset,
 * which exceeds SIM_TIELOG_CAP when records were dropped.  Waits for the
 * stream.  (SIM_E_STATE without SIM_F_TIELOG.) */
SIM_API int sim_tielog(sim_handle* h, sim_tie* out, int64_t capacity, int64_t* count);

/* Counters accumulated since the last reset with SIM_F_STATS (host array of
 * 4): processed tiles, ignition + continue trials, ignition trials with
 * |draw - p_ignite| <= 1e-5, launches. */
SIM_API int sim_stats(sim_handle* h, uint64_t out[4]);

/* Last error message of `h` (or of the last failed sim_init when h is NULL). */
SIM_API const char* sim_last_error(const sim_handle* h);

/* Release the handle (host memory only; the caller frees the workspace).  A
 * handle from sim_init_static first waits for its stream, then gives the
 * device's static scratch back. */
SIM_API void sim_destroy(sim_handle* h);

/* Library version string. */
SIM_API const char* sim_version(void);

#ifdef __cplusplus
}
#endif

#endif
