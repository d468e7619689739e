/*
 * fireoracle.c -- plain FP64 CPU oracle of the wildfire cellular automaton.
 *
 * TEST INFRASTRUCTURE ONLY (see fireoracle.h).  Deliberately slow and
 * literal: one cell at a time, one neighbour at a time, no blocking, no
 * reuse of partial results across cells or steps.
 *
 * Readings of passages the paper leaves open (all listed in the design
 * notes):
 *   - out-of-grid neighbours are not burning (hard edge);
 *   - p_veg, p_den, wind speed and wind direction are those of the receiving
 *     cell j; slope is atan((E_j - E_i)/(k l)) so uphill spread is positive;
 *   - the wind direction is the heading the wind blows toward, degrees
 *     counter-clockwise from east; the spread direction of i -> j is
 *     atan2(north, east) with east = -dc and north = +dr (rows run south);
 *   - f_p's constant is the FP32 rounding of 1.1486328125 (passed in `c`);
 *   - the two uniform matrices are Philox4x32-10 words 0 and 1 with counter
 *     (cell, 0, step, scenario) and key = seed;
 *   - a burnable cell ignites iff u < p_ignite, the comparison taken in FP32
 *     (the paper's working precision) on both sides: u < (float)p;
 *   - a burning cell stays burning iff u_cont < p_continue.
 */
#include "fireoracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- Philox */

/* One Philox4x32 round: two 32x32->64 products, the word permutation and
 * key xor of the Philox S-box (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 4). */
static void philox_round(uint32_t x[4], const uint32_t k[2])
{
    const uint64_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint64_t p0 = m0 * (uint64_t)x[0];
    uint64_t p1 = m1 * (uint64_t)x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x[1] ^ k[0];
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x[3] ^ k[1];
    uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}

void fo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {          /* Weyl key schedule between rounds */
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(x, k);
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

void fo_draws(const fo_problem* pb, int32_t t, int64_t cell, double* u_ign, double* u_cont)
{
    uint32_t ctr[4] = {(uint32_t)cell, (uint32_t)((uint64_t)cell >> 32), (uint32_t)t,
                       pb->scenario};
    uint32_t key[2] = {(uint32_t)pb->seed, (uint32_t)(pb->seed >> 32)};
    uint32_t r[4];
    fo_philox4x32_10(ctr, key, r);
    const double two_m24 = 1.0 / 16777216.0;
    if (u_ign) *u_ign = (double)(r[0] >> 8) * two_m24;
    if (u_cont) *u_cont = (double)(r[1] >> 8) * two_m24;
}

/* ------------------------------------------------------------ Eq. 1 - 5 */

static double wind_speed(const fo_problem* pb, int64_t j)
{
    return pb->wind_speed ? (double)pb->wind_speed[j] : pb->wind_speed_scalar;
}

static double wind_dir(const fo_problem* pb, int64_t j)
{
    return pb->wind_dir ? (double)pb->wind_dir[j] : pb->wind_dir_scalar;
}

/* Quantities of one edge i -> j, kept separate so the gradient can reuse the
 * exact same definitions. */
typedef struct {
    double F;        /* (1 + p_veg)(1 + p_den) of the receiving cell */
    double V;        /* wind speed at the receiving cell */
    double cosd;     /* cos(theta_w - phi) */
    double theta_s;  /* Eq. 1, degrees */
    double pw, ps;   /* Eq. 3, Eq. 4 */
    double x;        /* p_propagate of Eq. 2 */
    double q;        /* f_p(x) of Eq. 5 */
} fo_edge;

static void edge_eval(const fo_problem* pb, int32_t r, int32_t c, int32_t dr, int32_t dc,
                      fo_edge* e)
{
    const int64_t W = pb->W;
    const int64_t j = (int64_t)r * W + c;
    const int64_t i = (int64_t)(r + dr) * W + (c + dc);

    /* Eq. 1: slope between the receiving cell j and the burning neighbour i
     * (or the given slope tensor, the paper's own input form). */
    if (pb->slope9) {
        e->theta_s = (double)pb->slope9[j * 9 + (dr + 1) * 3 + (dc + 1)];
    } else {
        double k = (dr != 0 && dc != 0) ? sqrt(2.0) : 1.0;
        double Ej = (double)pb->elev[j];
        double Ei = (double)pb->elev[i];
        e->theta_s = atan((Ej - Ei) / (k * pb->cell_m)) * (180.0 / M_PI);
    }

    /* Eq. 3: theta_w is the angle between the wind heading and the spread
     * direction i -> j. */
    e->V = wind_speed(pb, j);
    double heading = wind_dir(pb, j) * (M_PI / 180.0);
    double phi = atan2((double)dr, (double)(-dc));
    e->cosd = cos(heading - phi);
    e->pw = exp(pb->c1 * e->V) * exp(pb->c2 * e->V * (e->cosd - 1.0));

    /* Eq. 4 */
    e->ps = exp(pb->a * e->theta_s);

    /* Eq. 2 */
    e->F = (1.0 + (double)pb->p_veg[j]) * (1.0 + (double)pb->p_den[j]);
    e->x = pb->p_h * e->F * e->pw * e->ps;

    /* Eq. 5 */
    e->q = tanh(pb->c * e->x);
}

double fo_edge_q(const fo_problem* pb, int32_t r, int32_t c, int32_t dr, int32_t dc,
                 double* theta_s_out, double* cosd_out)
{
    fo_edge e;
    edge_eval(pb, r, c, dr, dc, &e);
    if (theta_s_out) *theta_s_out = e.theta_s;
    if (cosd_out) *cosd_out = e.cosd;
    return e.q;
}

void fo_slope_tensor(const fo_problem* pb, float* out9)
{
    for (int32_t r = 0; r < pb->H; ++r)
        for (int32_t c = 0; c < pb->W; ++c)
            for (int32_t dr = -1; dr <= 1; ++dr)
                for (int32_t dc = -1; dc <= 1; ++dc) {
                    int64_t j = (int64_t)r * pb->W + c;
                    double v = 0.0;
                    int rr = r + dr, cc = c + dc;
                    if ((dr || dc) && rr >= 0 && rr < pb->H && cc >= 0 && cc < pb->W) {
                        double k = (dr != 0 && dc != 0) ? sqrt(2.0) : 1.0;
                        double Ei = (double)pb->elev[(int64_t)rr * pb->W + cc];
                        v = atan(((double)pb->elev[j] - Ei) / (k * pb->cell_m)) * (180.0 / M_PI);
                    }
                    out9[j * 9 + (dr + 1) * 3 + (dc + 1)] = (float)v;
                }
}

static int burning_at(const fo_problem* pb, const uint8_t* S, int32_t r, int32_t c)
{
    if (r < 0 || r >= pb->H || c < 0 || c >= pb->W) return 0;   /* hard edge */
    return S[(int64_t)r * pb->W + c] == 1;
}

/* ------------------------------------------------------------------ Eq. 9 */

double fo_pignite_cell(const fo_problem* pb, const uint8_t* S, int32_t r, int32_t c)
{
    if (S[(int64_t)r * pb->W + c] != 0) return 0.0;
    double prod = 1.0;
    for (int32_t dr = -1; dr <= 1; ++dr)
        for (int32_t dc = -1; dc <= 1; ++dc) {
            if (dr == 0 && dc == 0) continue;
            if (!burning_at(pb, S, r + dr, c + dc)) continue;
            fo_edge e;
            edge_eval(pb, r, c, dr, dc, &e);
            prod *= (1.0 - e.q);
        }
    return 1.0 - prod;
}

void fo_pignite_map(const fo_problem* pb, const uint8_t* S, double* out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t r = 0; r < pb->H; ++r)
        for (int32_t c = 0; c < pb->W; ++c)
            out[(int64_t)r * pb->W + c] = fo_pignite_cell(pb, S, r, c);
}

/* d p_ignite / d theta with theta = (p_h, a, c1, c2):
 *   dP/dq_i      = prod_{m != i} (1 - q_m)
 *   dq/dx        = c (1 - q^2)
 *   dx/dp_h      = F pw ps
 *   dx/da        = x theta_s
 *   dx/dc1       = x V
 *   dx/dc2       = x V (cos(delta) - 1)                                    */
void fo_dpignite_cell(const fo_problem* pb, const uint8_t* S, int32_t r, int32_t c,
                      double g[4])
{
    g[0] = g[1] = g[2] = g[3] = 0.0;
    if (S[(int64_t)r * pb->W + c] != 0) return;
    fo_edge e[8];
    int n = 0;
    for (int32_t dr = -1; dr <= 1; ++dr)
        for (int32_t dc = -1; dc <= 1; ++dc) {
            if (dr == 0 && dc == 0) continue;
            if (!burning_at(pb, S, r + dr, c + dc)) continue;
            edge_eval(pb, r, c, dr, dc, &e[n++]);
        }
    for (int i = 0; i < n; ++i) {
        double others = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != i) others *= (1.0 - e[m].q);
        double dqdx = pb->c * (1.0 - e[i].q * e[i].q);
        double s = others * dqdx;
        g[0] += s * e[i].F * e[i].pw * e[i].ps;
        g[1] += s * e[i].x * e[i].theta_s;
        g[2] += s * e[i].x * e[i].V;
        g[3] += s * e[i].x * e[i].V * (e[i].cosd - 1.0);
    }
}

/* --------------------------------------------------------------- stepping */

static int has_burning_neighbour(const fo_problem* pb, const uint8_t* S, int32_t r, int32_t c)
{
    for (int32_t dr = -1; dr <= 1; ++dr)
        for (int32_t dc = -1; dc <= 1; ++dc)
            if ((dr || dc) && burning_at(pb, S, r + dr, c + dc)) return 1;
    return 0;
}

uint8_t fo_next_cell(const fo_problem* pb, int32_t t, const uint8_t* S_prev, int32_t r,
                     int32_t c, double* p_out, int* tie_out, double tie_eps)
{
    const int64_t j = (int64_t)r * pb->W + c;
    const uint8_t s = S_prev[j];
    uint8_t next;
    double p = 0.0;
    int tie = 0;
    if (s == 2) {                     /* burned is absorbing */
        next = 2;
    } else if (s == 1) {              /* keep burning w.p. p_continue */
        double u_cont;
        fo_draws(pb, t, j, NULL, &u_cont);
        next = (u_cont < pb->p_continue) ? 1 : 2;
    } else if (!has_burning_neighbour(pb, S_prev, r, c)) {
        next = 0;                     /* no trial without a burning neighbour */
    } else {
        double u_ign;
        p = fo_pignite_cell(pb, S_prev, r, c);
        fo_draws(pb, t, j, &u_ign, NULL);
        next = (u_ign < (double)(float)p) ? 1 : 0;
        /* A near tie is a trial whose decision a different rounding of
         * p_ignite could change.  Without fuel at j, or with p_h = 0, every
         * edge has x = 0 exactly (Eq. 2), so p_ignite is exactly 0 in any
         * precision and the trial can never succeed: not a tie. */
        const double F = (1.0 + (double)pb->p_veg[j]) * (1.0 + (double)pb->p_den[j]);
        tie = F > 0.0 && pb->p_h > 0.0 && fabs(u_ign - p) <= tie_eps;
    }
    if (p_out) *p_out = p;
    if (tie_out) *tie_out = tie;
    return next;
}

int64_t fo_step(const fo_problem* pb, int32_t t, const uint8_t* S_prev, uint8_t* S_next,
                double* yhat, uint8_t* tie, double tie_eps, double* pmap)
{
    int64_t ties = 0;
    /* Cells are independent within a step (every rule reads S(t-1) only), so
     * the threaded build splits the rows; the per-cell arithmetic is the same
     * in both builds. */
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : ties)
    for (int32_t r = 0; r < pb->H; ++r)
        for (int32_t c = 0; c < pb->W; ++c) {
            const int64_t j = (int64_t)r * pb->W + c;
            double p;
            int tj;
            S_next[j] = fo_next_cell(pb, t, S_prev, r, c, &p, &tj, tie_eps);
            if (S_prev[j] == 0 && S_next[j] == 1 && yhat) yhat[j] = p;
            ties += tj;
            if (tie) tie[j] = (uint8_t)tj;
            if (pmap) pmap[j] = p;
        }
    return ties;
}

int64_t fo_run(const fo_problem* pb, int32_t t0, int32_t T, uint8_t* S, double* yhat,
               int32_t* tstep, double tie_eps)
{
    return fo_run_ties(pb, t0, T, S, yhat, tstep, tie_eps, NULL, NULL, 0);
}

int64_t fo_run_ties(const fo_problem* pb, int32_t t0, int32_t T, uint8_t* S, double* yhat,
                    int32_t* tstep, double tie_eps, int32_t* tie_step, int64_t* tie_cell,
                    int64_t cap)
{
    const int64_t n = (int64_t)pb->H * pb->W;
    uint8_t* nxt = (uint8_t*)malloc((size_t)n);
    uint8_t* tie = cap > 0 ? (uint8_t*)calloc((size_t)n, 1) : NULL;
    int64_t ties = 0;
    for (int32_t t = t0 + 1; t <= t0 + T; ++t) {
        const int64_t k = fo_step(pb, t, S, nxt, yhat, tie, tie_eps, NULL);
        if (tie && k > 0) {
            /* list this step's near ties in cell order */
            int64_t found = 0;
            for (int64_t j = 0; j < n && found < k; ++j)
                if (tie[j]) {
                    if (ties + found < cap) {
                        tie_step[ties + found] = t;
                        tie_cell[ties + found] = j;
                    }
                    ++found;
                }
        }
        ties += k;
        if (tstep)
            for (int64_t j = 0; j < n; ++j)
                if (S[j] == 0 && nxt[j] == 1) tstep[j] = t;
        memcpy(S, nxt, (size_t)n);
    }
    free(tie);
    free(nxt);
    return ties;
}

int fo_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ----------------------------------------------------------------- Eq. 10 */

double fo_loss(int32_t H, int32_t W, const double* yhat, const uint8_t* y, int32_t kind,
               double* lambda)
{
    const int64_t n = (int64_t)H * W;
    if (lambda)
        for (int64_t j = 0; j < n; ++j) lambda[j] = 0.0;
    double loss = 0.0;

    if (kind == 0 || kind == 1) {
        /* BCE-with-logits over the bounding box of (yhat != 0) | (y != 0). */
        int32_t r0 = H, r1 = -1, c0 = W, c1 = -1;
        for (int32_t r = 0; r < H; ++r)
            for (int32_t c = 0; c < W; ++c) {
                int64_t j = (int64_t)r * W + c;
                if (yhat[j] != 0.0 || y[j] != 0) {
                    if (r < r0) r0 = r;
                    if (r > r1) r1 = r;
                    if (c < c0) c0 = c;
                    if (c > c1) c1 = c;
                }
            }
        if (r1 >= 0) {
            double N = (double)(r1 - r0 + 1) * (double)(c1 - c0 + 1);
            double s = 0.0;
            for (int32_t r = r0; r <= r1; ++r)
                for (int32_t c = c0; c <= c1; ++c) {
                    int64_t j = (int64_t)r * W + c;
                    double z = yhat[j], yy = (double)y[j];
                    double sig = 1.0 / (1.0 + exp(-z));
                    s += -(yy * log(sig) + (1.0 - yy) * log(1.0 - sig));
                    if (lambda) lambda[j] += (sig - yy) / N;
                }
            loss += s / N;
        }
    }
    if (kind == 1 || kind == 2) {
        /* Squared difference of 4x4 / stride-4 average pools (floor mode). */
        int32_t Hp = H / 4, Wp = W / 4;
        if (Hp > 0 && Wp > 0) {
            double Np = (double)Hp * (double)Wp;
            double s = 0.0;
            for (int32_t pr = 0; pr < Hp; ++pr)
                for (int32_t pc = 0; pc < Wp; ++pc) {
                    double a = 0.0, b = 0.0;
                    for (int32_t dr = 0; dr < 4; ++dr)
                        for (int32_t dc = 0; dc < 4; ++dc) {
                            int64_t j = (int64_t)(4 * pr + dr) * W + (4 * pc + dc);
                            a += yhat[j];
                            b += (double)y[j];
                        }
                    double d = a / 16.0 - b / 16.0;
                    s += d * d;
                    if (lambda)
                        for (int32_t dr = 0; dr < 4; ++dr)
                            for (int32_t dc = 0; dc < 4; ++dc) {
                                int64_t j = (int64_t)(4 * pr + dr) * W + (4 * pc + dc);
                                lambda[j] += 2.0 * d / (16.0 * Np);
                            }
                }
            loss += s / Np;
        }
    }
    return loss;
}

/* ------------------------------------------------------- analytic gradient */

void fo_grad(const fo_problem* pb, int32_t T, const uint8_t* S_init, const double* lambda,
             double g[4])
{
    const int64_t n = (int64_t)pb->H * pb->W;
    uint8_t* S = (uint8_t*)malloc((size_t)n);
    uint8_t* nxt = (uint8_t*)malloc((size_t)n);
    for (int64_t j = 0; j < n; ++j) S[j] = S_init[j] ? 1 : 0;
    g[0] = g[1] = g[2] = g[3] = 0.0;
    for (int32_t t = 1; t <= T; ++t) {
        fo_step(pb, t, S, nxt, NULL, NULL, 0.0, NULL);
        for (int32_t r = 0; r < pb->H; ++r)
            for (int32_t c = 0; c < pb->W; ++c) {
                int64_t j = (int64_t)r * pb->W + c;
                if (S[j] == 0 && nxt[j] == 1) {
                    double d[4];
                    fo_dpignite_cell(pb, S, r, c, d);
                    for (int k = 0; k < 4; ++k) g[k] += lambda[j] * d[k];
                }
            }
        memcpy(S, nxt, (size_t)n);
    }
    free(S);
    free(nxt);
}
