/*
 * fireoracle.h -- plain FP64 CPU oracle of the wildfire cellular automaton.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * never links, calls or shares code with it.
 *
 * It follows "PyTorchFire: A GPU-Accelerated Wildfire Simulator with
 * Differentiable Cellular Automata" (Xia & Cheng, 2025):
 *   Sec. 2.1  inputs / outputs / parameters, Eq. 1 (slope from elevation)
 *   Sec. 2.2  state and transition rules, Eq. 2-5 (propagation and f_p),
 *             Eq. 9 (ignition probability), the data-flow paragraph
 *             (two uniform random matrices, accumulator of newly ignited
 *             p_ignite)
 *   Sec. 2.3  Eq. 10 (loss), step rings (gradient only through p_ignite of
 *             ignited cells)
 *
 * Every routine reads the same FP32 inputs the GPU receives, widened to
 * double, and computes in double.  State codes: 0 burnable, 1 burning,
 * 2 burned.  Arrays are row-major H x W, row 0 = north, columns run east.
 *
 * Pin status (tests/test_oracle_pins.py):
 *   fo_philox4x32_10      pinned (published known-answer vectors, rocRAND's
 *                         header-only engine, uniformity)
 *   fo_edge_q             pinned (closed forms: calm/flat/neutral, wind
 *                         directions, slope angles incl. diagonal, fuel)
 *   fo_pignite_cell/map   pinned (binomial closed form, brute-force
 *                         enumeration, 90/180 degree rotation covariance)
 *   fo_step / fo_run      pinned (3x3 exact next-state distribution vs
 *                         Monte-Carlo over seeds, invariants)
 *   fo_dpignite_cell,
 *   fo_grad               pinned (FP64 central finite differences with
 *                         common random numbers; vanishing-derivative cases)
 *   fo_loss               pinned (closed forms on hand-made maps; finite
 *                         differences of the loss for lambda)
 *   fo_slope_tensor       pinned (hand-computed 45 degree edges, sign and
 *                         layout; equivalence with the elevation path)
 */
#ifndef FIREORACLE_H
#define FIREORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t H, W;
    double cell_m;                 /* l of Eq. 1, metres */
    uint64_t seed;                 /* Philox key */
    uint32_t scenario;             /* Philox counter word 3 */
    double p_h, a, c1, c2, p_continue;
    double c;                      /* f_p constant of Eq. 5 */
    const float *p_veg, *p_den, *elev;       /* H*W */
    const float *wind_speed, *wind_dir;      /* H*W, or NULL -> scalars */
    double wind_speed_scalar, wind_dir_scalar;
    const float *slope9;           /* H*W*3*3 degrees (paper layout) or NULL -> Eq. 1 */
} fo_problem;

/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 S-box. */
void fo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The two uniforms of cell `cell` at step t: u_ign from word 0, u_cont from
 * word 1, each (w >> 8) * 2^-24. */
void fo_draws(const fo_problem* pb, int32_t t, int64_t cell, double* u_ign, double* u_cont);

/* f_p(p_propagate) of Eq. 2-5 for a burning neighbour at (r+dr, c+dc)
 * spreading into cell (r, c); both cells must lie inside the grid (cells
 * outside it never burn).  Optional outputs: theta_s (deg), cos(delta). */
double fo_edge_q(const fo_problem* pb, int32_t r, int32_t c, int32_t dr, int32_t dc,
                 double* theta_s_out, double* cosd_out);

/* Eq. 1 angles in the paper's slope-tensor layout: out9[(r*W + c)*9 +
 * (dr+1)*3 + (dc+1)] = angle (degrees, FP32) of the edge from the neighbour
 * (r+dr, c+dc) into (r, c); 0 for the centre and out-of-grid slots.  Needs
 * pb->elev.  Feeding the result back as pb->slope9 reproduces the
 * elevation-based model up to the FP32 rounding of the angles. */
void fo_slope_tensor(const fo_problem* pb, float* out9);

/* Eq. 9 for cell (r, c) of state S; 0 for cells that are not burnable. */
double fo_pignite_cell(const fo_problem* pb, const uint8_t* S, int32_t r, int32_t c);
void fo_pignite_map(const fo_problem* pb, const uint8_t* S, double* out);

/* d p_ignite / d(p_h, a, c1, c2) at cell (r, c) of state S. */
void fo_dpignite_cell(const fo_problem* pb, const uint8_t* S, int32_t r, int32_t c,
                      double g[4]);

/* The state at step t of cell (r, c) from S(t-1) = S_prev (the per-cell rule
 * of fo_step).  p_out (nullable) receives p_ignite for ignition trials, else 0;
 * tie_out (nullable) 1 for an ignition trial with |u - p| <= tie_eps whose
 * receiving cell has fuel (with p_h > 0): trials at cells without fuel have
 * p_ignite exactly 0 in any precision and are never near ties. */
uint8_t fo_next_cell(const fo_problem* pb, int32_t t, const uint8_t* S_prev, int32_t r,
                     int32_t c, double* p_out, int* tie_out, double tie_eps);

/* One synchronous step producing S(t) from S(t-1) = S_prev.
 *   yhat  (nullable): p_ignite written for cells that ignite at this step
 *   tie   (nullable): set to 1 for ignition trials with |u - p| <= tie_eps
 *   pmap  (nullable): p_ignite of every cell for S_prev
 * Returns the number of near-tie ignition trials. */
int64_t fo_step(const fo_problem* pb, int32_t t, const uint8_t* S_prev, uint8_t* S_next,
                double* yhat, uint8_t* tie, double tie_eps, double* pmap);

/* Steps t0+1 .. t0+T starting from S (uint8 {0,1,2}), in place.  yhat
 * (nullable) accumulates as in fo_step.  tstep (nullable, int32 H*W) receives
 * the step at which each cell ignites.  Returns the near-tie count. */
int64_t fo_run(const fo_problem* pb, int32_t t0, int32_t T, uint8_t* S, double* yhat,
               int32_t* tstep, double tie_eps);

/* fo_run that also lists its near ties: the first `cap` of them in step and
 * cell order go to tie_step[k] / tie_cell[k] (nullable when cap is 0).
 * Returns the near-tie count (which may exceed cap). */
int64_t fo_run_ties(const fo_problem* pb, int32_t t0, int32_t T, uint8_t* S, double* yhat,
                    int32_t* tstep, double tie_eps, int32_t* tie_step, int64_t* tie_cell,
                    int64_t cap);

/* Threads of the row loops in fo_step / fo_pignite_map when the library is
 * built with OpenMP (liboracle_omp.so): sets the count when n > 0 and returns
 * the count in use (always 1 in the plain build). */
int fo_threads(int n);

/* Eq. 10: loss_kind 0 = BCE-with-logits on the bounding-box crop of
 * (yhat != 0) | (y != 0); 1 = BCE + MSE of 4x4 average pools; 2 = MSE only.
 * lambda (nullable) receives dL/dyhat. */
double fo_loss(int32_t H, int32_t W, const double* yhat, const uint8_t* y, int32_t kind,
               double* lambda);

/* Gradient of sum_j lambda_j * yhat_j over the run from S_init (burning
 * cells = 1), with states held constant (gradient only through p_ignite of
 * the cells that ignite). */
void fo_grad(const fo_problem* pb, int32_t T, const uint8_t* S_init, const double* lambda,
             double g[4]);

#ifdef __cplusplus
}
#endif

#endif
