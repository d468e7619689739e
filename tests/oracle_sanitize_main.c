/* Drives every entry point of the C oracle on small grids, so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer can catch an
 * out-of-bounds access, an uninitialised read or undefined arithmetic in
 * it.  Test support only (built by tests/test_oracle_sanitizers.py); exits
 * non-zero when an invariant of the automaton fails. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fireoracle.h"

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static double urand(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int fail(const char* what, int H, int W) {
    fprintf(stderr, "FAIL %s (H=%d W=%d)\n", what, H, W);
    return 1;
}

static int run_case(int H, int W, int per_cell_wind, int use_slope9, int T) {
    const int64_t n = (int64_t)H * W;
    float* veg = malloc(sizeof(float) * n);
    float* den = malloc(sizeof(float) * n);
    float* el = malloc(sizeof(float) * n);
    float* ws = malloc(sizeof(float) * n);
    float* wd = malloc(sizeof(float) * n);
    float* s9 = malloc(sizeof(float) * 9 * n);
    uint8_t* S = malloc(n);
    uint8_t* S0 = malloc(n);
    uint8_t* S1 = malloc(n);
    uint8_t* tie = malloc(n);
    uint8_t* y = malloc(n);
    double* yhat = calloc(n, sizeof(double));
    double* pmap = malloc(sizeof(double) * n);
    double* lam = malloc(sizeof(double) * n);
    int32_t* tstep = malloc(sizeof(int32_t) * n);
    int32_t tie_step[16];
    int64_t tie_cell[16];
    int bad = 0;
    for (int64_t j = 0; j < n; ++j) {
        veg[j] = urand() < 0.1 ? -1.f : (float)(urand() * 0.7 - 0.3);
        den[j] = (float)(urand() * 0.7 - 0.4);
        el[j] = (float)(urand() * 60.0);
        ws[j] = (float)(urand() * 12.0);
        wd[j] = (float)(urand() * 360.0);
        S[j] = 0;
    }
    S[(H / 2) * (int64_t)W + W / 2] = 1;
    veg[(H / 2) * (int64_t)W + W / 2] = 0.f;
    fo_problem pb;
    memset(&pb, 0, sizeof pb);
    pb.H = H;
    pb.W = W;
    pb.cell_m = 30.0;
    pb.seed = 12345;
    pb.scenario = 7;
    pb.p_h = 0.58;
    pb.a = 0.078;
    pb.c1 = 0.045;
    pb.c2 = 0.131;
    pb.p_continue = 0.3;
    pb.c = (double)1.1486328125f;
    pb.p_veg = veg;
    pb.p_den = den;
    pb.elev = el;
    pb.wind_speed = per_cell_wind ? ws : NULL;
    pb.wind_dir = per_cell_wind ? wd : NULL;
    pb.wind_speed_scalar = 5.0;
    pb.wind_dir_scalar = 45.0;
    fo_slope_tensor(&pb, s9);
    if (use_slope9) pb.slope9 = s9;

    memcpy(S0, S, n);
    for (int32_t r = 0; r < H; ++r)
        for (int32_t c = 0; c < W; ++c)
            for (int dr = -1; dr <= 1; ++dr)
                for (int dc = -1; dc <= 1; ++dc) {
                    if (!dr && !dc) continue;
                    // only neighbours inside the grid can burn
                    if (r + dr < 0 || r + dr >= H || c + dc < 0 || c + dc >= W) continue;
                    double th = 0, cd = 0;
                    const double q = fo_edge_q(&pb, r, c, dr, dc, &th, &cd);
                    if (!(q >= 0.0 && q <= 1.0)) bad |= fail("edge q outside [0, 1]", H, W);
                }
    for (int t = 1; t <= T; ++t) {
        fo_pignite_map(&pb, S, pmap);
        const int64_t ties = fo_step(&pb, t, S, S1, yhat, tie, 1e-5, pmap);
        if (ties < 0) bad |= fail("negative tie count", H, W);
        for (int64_t j = 0; j < n; ++j) {
            if (S1[j] > 2) bad |= fail("state code", H, W);
            if (S[j] == 2 && S1[j] != 2) bad |= fail("burned cell changed", H, W);
            if (S1[j] == 1 && S[j] == 0 && !(pmap[j] > 0.0)) bad |= fail("ignition with p = 0", H, W);
            double g[4];
            const int32_t r = (int32_t)(j / W), c = (int32_t)(j % W);
            double p = 0;
            int tf = 0;
            (void)fo_next_cell(&pb, t, S, r, c, &p, &tf, 1e-5);
            if (S[j] == 0) fo_dpignite_cell(&pb, S, r, c, g);
        }
        memcpy(S, S1, n);
    }
    for (int64_t j = 0; j < n; ++j) y[j] = S[j] != 0;
    for (int kind = 0; kind < 3; ++kind) {
        const double L = fo_loss(H, W, yhat, y, kind, lam);
        if (!isfinite(L)) bad |= fail("loss not finite", H, W);
    }
    double g[4];
    fo_grad(&pb, T, S0, lam, g);
    for (int k = 0; k < 4; ++k)
        if (!isfinite(g[k])) bad |= fail("gradient not finite", H, W);
    memcpy(S, S0, n);
    (void)fo_run(&pb, 0, T, S, yhat, tstep, 1e-5);
    memcpy(S, S0, n);
    (void)fo_run_ties(&pb, 0, T, S, yhat, tstep, 1e-5, tie_step, tie_cell, 16);
    memcpy(S, S0, n);
    (void)fo_run_ties(&pb, 0, T, S, NULL, NULL, 1e-5, NULL, NULL, 0);
    double u0, u1;
    fo_draws(&pb, 1, n - 1, &u0, &u1);
    if (!(u0 >= 0 && u0 < 1 && u1 >= 0 && u1 < 1)) bad |= fail("draw outside [0, 1)", H, W);
    free(veg); free(den); free(el); free(ws); free(wd); free(s9); free(S); free(S0);
    free(S1); free(tie); free(y); free(yhat); free(pmap); free(lam); free(tstep);
    return bad;
}

int main(void) {
    const int cases[][5] = {
        {1, 1, 0, 0, 3}, {1, 37, 1, 0, 20}, {29, 1, 0, 1, 20}, {2, 2, 1, 1, 5},
        {17, 23, 1, 0, 30}, {33, 31, 0, 1, 30}, {40, 64, 1, 1, 25},
    };
    int bad = 0;
    for (size_t i = 0; i < sizeof cases / sizeof cases[0]; ++i)
        bad |= run_case(cases[i][0], cases[i][1], cases[i][2], cases[i][3], cases[i][4]);
    fo_threads(0);
    printf(bad ? "oracle sanitizer run: FAILED\n" : "oracle sanitizer run: ok\n");
    return bad;
}
