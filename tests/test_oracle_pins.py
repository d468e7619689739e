"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these checks re-evaluates the oracle's own expressions: each one uses
a special case with a closed form, an exact enumeration, a published
known-answer vector, an independent implementation (rocRAND's header-only
Philox engine), an invariant of the transition rules, or finite differences.
"""

import dataclasses
import json
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))
C = float(np.float32(GOLDEN["c_normaliser"]["value"]))


def flat_scenario(H, W, *, veg=0.0, den=0.0, elev=0.0, V=0.0, theta=0.0, cell_m=30.0,
                  p=(0.58, 0.078, 0.045, 0.131, 0.3), seed=7, scenario_id=0):
    f = lambda v: np.full((H, W), v, dtype=np.float32)
    s = synth.Scenario(H=H, W=W, p_veg=f(veg), p_den=f(den), elevation=f(elev),
                       wind_speed=None, wind_dir=None, wind_speed_scalar=V,
                       wind_dir_scalar=theta, init_burning=np.zeros((H, W), np.uint8),
                       cell_m=cell_m, seed=seed, scenario_id=scenario_id)
    return s.with_params(*p)


NEIGHBOURS = [(dr, dc) for dr in (-1, 0, 1) for dc in (-1, 0, 1) if (dr, dc) != (0, 0)]


# --------------------------------------------------------------- Eq. 5 / 8

def test_normaliser_constant_from_nelder_mead():
    """Sec. 2.2: tanh(cx) fitted to y = x on [0.2, 0.8] by Nelder-Mead gives c."""
    from scipy.optimize import minimize
    xs = np.linspace(0.2, 0.8, 100)
    cands = {
        "eq6": lambda c, x: -c ** (-x) + 1.0,
        "eq7": lambda c, x: -(x + 1.0) ** (-c) + 1.0,
        "eq8": lambda c, x: np.tanh(c * x),
    }
    sse = {}
    best = {}
    for k, f in cands.items():
        res = minimize(lambda c: np.sum((f(c[0], xs) - xs) ** 2), x0=[1.0],
                       method="Nelder-Mead")
        best[k], sse[k] = float(res.x[0]), float(res.fun)
    assert abs(best["eq8"] - GOLDEN["c_normaliser"]["value"]) < 1e-12
    assert sse["eq8"] < sse["eq6"] and sse["eq8"] < sse["eq7"]
    import oracle
    assert oracle.C_F32 == C


# ------------------------------------------------------------------ Philox

KAT = [  # Random123 known-answer vectors for philox4x32_10
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(oracle_lib, ctr, key, want):
    assert list(oracle_lib.philox4x32_10(ctr, key)) == want


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    unsigned long long seed = strtoull(argv[a], 0, 0);
    unsigned long long sub = strtoull(argv[a + 1], 0, 0);
    unsigned long long off = strtoull(argv[a + 2], 0, 0);
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    for (int i = 0; i < 4; ++i) printf("%u\n", e());
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_header(oracle_lib):
    """The oracle's counter layout (cell, 0, step, scenario) equals rocRAND's
    (offset / 4, subsequence) layout; its engine is an independent code."""
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(6):
        seed = int(rng.integers(0, 2**63))
        cell = int(rng.integers(0, 2**31))
        t = int(rng.integers(0, 5000))
        scen = int(rng.integers(0, 300))
        cases.append((seed, cell, t, scen))
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "p.cpp"), os.path.join(d, "p")
        open(src, "w").write(ROCRAND_PROBE)
        subprocess.check_call(["hipcc", "-O1", "-o", exe, src],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        args = []
        for seed, cell, t, scen in cases:
            args += [str(seed), str(t | (scen << 32)), str(4 * cell)]
        out = subprocess.check_output([exe] + args).decode().split()
    got = np.array([int(x) for x in out], dtype=np.uint64).reshape(-1, 4)
    for (seed, cell, t, scen), ref in zip(cases, got):
        mine = oracle_lib.philox4x32_10([cell, 0, t, scen], [seed & 0xFFFFFFFF, seed >> 32])
        assert list(mine) == list(ref)


def test_draws_uniform_on_2m24_grid(oracle_lib):
    s = flat_scenario(4, 4, seed=123456789)
    us = np.array([oracle_lib.draws(s, t, cell) for t in range(1, 41)
                   for cell in range(0, 5000, 1)])
    assert np.all(us >= 0) and np.all(us < 1)
    assert np.all(us * 2**24 == np.round(us * 2**24))
    for col in range(2):
        assert stats.kstest(us[:, col], "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(us[:, 0], us[:, 1])[0, 1]) < 0.01


# ---------------------------------------------------------- Eq. 2 - 5, 9

def test_calm_flat_neutral_binomial(oracle_lib):
    """Calm, flat, neutral fuel: every edge has q0 = tanh(c p_h) and Eq. 9
    reduces to 1 - (1 - q0)^n for all 256 burning-neighbour patterns."""
    s = flat_scenario(3, 3)
    q0 = math.tanh(C * float(np.float32(0.58)))
    for mask in range(256):
        S = np.zeros((3, 3), np.uint8)
        for k, (dr, dc) in enumerate(NEIGHBOURS):
            if mask >> k & 1:
                S[1 + dr, 1 + dc] = 1
        n = bin(mask).count("1")
        p = oracle_lib.pignite_cell(s, S, 1, 1)
        assert p == pytest.approx(1.0 - (1.0 - q0) ** n, rel=1e-14, abs=1e-16)


@pytest.mark.parametrize("theta", [0.0, 45.0, 90.0, 135.0, 200.0, 315.0])
def test_wind_direction_convention(oracle_lib, theta):
    """Eq. 3: spread straight downwind has cos = 1, upwind -1, across 0.
    Wind blows toward theta (deg CCW from east); row 0 is north."""
    V = 5.0
    s = flat_scenario(3, 3, V=V, theta=theta)
    ph, c1, c2 = (float(np.float32(v)) for v in (0.58, 0.045, 0.131))
    hx, hy = math.cos(math.radians(theta)), math.sin(math.radians(theta))
    for dr, dc in NEIGHBOURS:
        q, th, cosd = oracle_lib.edge_q(s, 1, 1, dr, dc)
        # the fire travels from (1+dr, 1+dc) to (1, 1): east = -dc, north = +dr
        east, north = -dc, dr
        norm = math.hypot(east, north)
        want = (east * hx + north * hy) / norm
        assert cosd == pytest.approx(want, abs=1e-12)
        assert th == 0.0
    # downwind special case: p_w = exp(c1 V) only
    dr = round(hy) if abs(hy) > 0.5 else 0    # north of travel = +dr
    dc = -round(hx) if abs(hx) > 0.5 else 0   # east of travel = -dc
    if theta in (0.0, 90.0):
        q, _, cosd = oracle_lib.edge_q(s, 1, 1, dr, dc)
        assert cosd == pytest.approx(1.0, abs=1e-15)
        assert q == pytest.approx(math.tanh(C * ph * math.exp(c1 * V)), rel=1e-14)
        q, _, _ = oracle_lib.edge_q(s, 1, 1, -dr, -dc)
        assert q == pytest.approx(math.tanh(C * ph * math.exp(c1 * V - 2 * c2 * V)), rel=1e-13)


def test_wind_45_orders_neighbours(oracle_lib):
    """Wind toward NE: the SW neighbour is downwind (largest q), NE upwind."""
    s = flat_scenario(3, 3, V=5.0, theta=45.0)
    q = {nb: oracle_lib.edge_q(s, 1, 1, *nb)[0] for nb in NEIGHBOURS}
    assert max(q, key=q.get) == (1, -1)
    assert min(q, key=q.get) == (-1, 1)
    assert q[(0, -1)] == pytest.approx(q[(1, 0)], rel=1e-14)
    assert q[(-1, -1)] == pytest.approx(q[(1, 1)], rel=1e-14)
    assert q[(-1, 0)] == pytest.approx(q[(0, 1)], rel=1e-14)


def test_slope_angles_and_diagonal_distance(oracle_lib):
    """Eq. 1/4: a neighbour l metres lower (adjacent) or l*sqrt2 lower
    (diagonal) gives exactly 45 deg uphill; l metres higher gives -45."""
    a = float(np.float32(0.078))
    ph = float(np.float32(0.58))
    l = 30.0
    for dr, dc in NEIGHBOURS:
        diag = dr != 0 and dc != 0
        drop = l * (math.sqrt(2.0) if diag else 1.0)
        E = np.zeros((3, 3), np.float32)
        E[1, 1] = 1000.0
        E[1 + dr, 1 + dc] = np.float32(1000.0 - drop)
        s = flat_scenario(3, 3, cell_m=l)
        s.elevation = E
        q, th, _ = oracle_lib.edge_q(s, 1, 1, dr, dc)
        exact_drop = 1000.0 - float(E[1 + dr, 1 + dc])
        want_th = math.degrees(math.atan(exact_drop / (l * (math.sqrt(2) if diag else 1))))
        assert th == pytest.approx(want_th, abs=1e-12)
        assert th == pytest.approx(45.0, abs=2e-3)
        assert q == pytest.approx(math.tanh(C * ph * math.exp(a * want_th)), rel=1e-13)
        E[1 + dr, 1 + dc] = np.float32(1000.0 + drop)
        q2, th2, _ = oracle_lib.edge_q(s, 1, 1, dr, dc)
        assert th2 < 0 and q2 < q


def test_fuel_factors(oracle_lib):
    ph = float(np.float32(0.58))
    for veg, den in [(0.4, 0.3), (-0.3, -0.4), (0.2, 0.0)]:
        s = flat_scenario(3, 3, veg=veg, den=den)
        q = oracle_lib.edge_q(s, 1, 1, 0, 1)[0]
        F = (1 + float(np.float32(veg))) * (1 + float(np.float32(den)))
        assert q == pytest.approx(math.tanh(C * ph * F), rel=1e-14)
    s = flat_scenario(3, 3, veg=-1.0, den=0.3)
    assert oracle_lib.edge_q(s, 1, 1, 0, 1)[0] == 0.0
    S = np.ones((3, 3), np.uint8)
    S[1, 1] = 0
    assert oracle_lib.pignite_cell(s, S, 1, 1) == 0.0


def random_small(H, W, seed, per_cell_wind=True):
    rng = np.random.default_rng(seed)
    s = synth.make_lakes(H, W, seed) if per_cell_wind else synth.make_plain(H, W, seed)
    S = rng.choice([0, 1, 2], size=(H, W), p=[0.5, 0.35, 0.15]).astype(np.uint8)
    return s, S


def test_bruteforce_edge_enumeration(oracle_lib):
    """Eq. 9 equals P(at least one of the independent edges fires), by
    enumerating all 2^n outcomes of the burning edges."""
    for seed in range(20):
        s, S = random_small(3, 3, seed)
        S[1, 1] = 0
        qs = [oracle_lib.edge_q(s, 1, 1, dr, dc)[0] for dr, dc in NEIGHBOURS
              if S[1 + dr, 1 + dc] == 1]
        p_any = 0.0
        for outcome in range(1 << len(qs)):
            pr = 1.0
            for k, q in enumerate(qs):
                pr *= q if outcome >> k & 1 else (1.0 - q)
            if outcome:
                p_any += pr
        assert oracle_lib.pignite_cell(s, S, 1, 1) == pytest.approx(p_any, abs=1e-14)


def test_next_state_distribution_3x3(oracle_lib):
    """One step on a 3x3 grid: the joint law of the 9 next states is the
    product of per-cell Bernoullis (p_ignite for burnable cells with a burning
    neighbour, p_continue for burning cells).  The oracle's seeded sampler
    must reproduce the exact enumerated law (chi-square, alpha = 1e-3)."""
    s, _ = random_small(3, 3, 3, per_cell_wind=True)
    S = np.array([[1, 0, 0], [0, 0, 2], [1, 0, 1]], np.uint8)
    pmap = oracle_lib.pignite_map(s, S)
    pc = float(np.float32(s.p_continue))
    trials = []  # (cell, prob of "burning next")
    for j in range(9):
        r, c = divmod(j, 3)
        if S[r, c] == 1:
            trials.append((j, pc))
        elif S[r, c] == 0 and pmap[r, c] > 0:
            trials.append((j, pmap[r, c]))
    m = len(trials)
    probs = np.zeros(1 << m)
    for o in range(1 << m):
        pr = 1.0
        for k, (_, p) in enumerate(trials):
            pr *= p if o >> k & 1 else 1 - p
        probs[o] = pr
    counts = np.zeros(1 << m)
    n = 20000
    for seed in range(n):
        nxt, _, _, _ = oracle_lib.step(s, 1, S, seed=seed * 7919 + 1)
        o = 0
        for k, (j, _) in enumerate(trials):
            o |= int(nxt.flat[j] == 1) << k
        counts[o] += 1
        assert np.all(nxt[S == 2] == 2)
        assert np.all(nxt[(S == 1) & (nxt != 1)] == 2)
    exp = probs * n
    keep = exp >= 5
    chi2 = np.sum((counts[keep] - exp[keep]) ** 2 / exp[keep])
    dof = keep.sum() - 1
    assert stats.chi2.sf(chi2, dof) > 1e-3
    assert counts[~keep].sum() <= max(10, 3 * exp[~keep].sum() + 10)


def test_rotation_covariance(oracle_lib):
    """Rotating every field by 90 deg counter-clockwise and turning the wind
    heading by +90 deg rotates the p_ignite map (pins the handedness of the
    grid/wind conventions)."""
    s, S = random_small(9, 7, 5, per_cell_wind=True)
    p0 = oracle_lib.pignite_map(s, S)
    for k in (1, 2, 3):
        r = synth.Scenario(H=s.W if k % 2 else s.H, W=s.H if k % 2 else s.W,
                           p_veg=np.rot90(s.p_veg, k).copy(),
                           p_den=np.rot90(s.p_den, k).copy(),
                           elevation=np.rot90(s.elevation, k).copy(),
                           wind_speed=np.rot90(s.wind_speed, k).copy(),
                           wind_dir=np.mod(np.rot90(s.wind_dir, k) + 90.0 * k,
                                           360.0).astype(np.float32),
                           wind_speed_scalar=0.0, wind_dir_scalar=0.0,
                           init_burning=np.rot90(s.init_burning, k).copy())
        r = r.with_params(*s.params)
        pr = oracle_lib.pignite_map(r, np.rot90(S, k).copy())
        np.testing.assert_allclose(pr, np.rot90(p0, k), rtol=1e-6, atol=1e-12)


# ------------------------------------------------------ transition invariants

def check_trajectory(oracle_lib, s, T):
    S = oracle_lib.initial_state(s)
    fuelless = s.p_veg <= -1.0
    ever = S == 1
    for t in range(1, T + 1):
        nxt, _, _, _ = oracle_lib.step(s, t, S)
        assert np.all(nxt[S == 2] == 2)                       # burned absorbing
        new = (S == 0) & (nxt == 1)
        pad = np.pad(S == 1, 1)
        nb = np.zeros_like(S, dtype=bool)
        for dr, dc in NEIGHBOURS:
            nb |= pad[1 + dr:1 + dr + s.H, 1 + dc:1 + dc + s.W]
        assert not np.any(new & ~nb)                          # needs a burning nbr
        assert not np.any(new & fuelless)                     # no fuel, no fire
        assert np.all(nxt[(S == 0) & ~nb] == 0)
        ever |= nxt == 1
        S = nxt
    return S, ever


def test_invariants_config0_like(oracle_lib):
    s = synth.make_plain(48, 40, 3, T=60)
    check_trajectory(oracle_lib, s, 60)


def test_wall_blocks_fire(oracle_lib):
    s = synth.make_plain(30, 30, 4, nonburn_frac=0.0, ignitions=[(15, 5)])
    s.p_veg = s.p_veg.copy()
    s.p_veg[:, 12] = -1.0
    s = s.with_params(1.0, 0.0, 0.0, 0.0, 0.5)
    S, ever = check_trajectory(oracle_lib, s, 80)
    assert ever[:, :12].sum() > 50
    assert not ever[:, 12:].any()


def test_parameter_extremes(oracle_lib):
    base = synth.make_plain(24, 24, 9, nonburn_frac=0.0)
    S0 = oracle_lib.initial_state(base)
    # p_h = 0: nothing spreads
    r = oracle_lib.run(base.with_params(p_h=0.0), 10)
    assert (r["S"] == 1).sum() + (r["S"] == 2).sum() == (S0 == 1).sum()
    # p_continue = 0: every cell burns exactly one step
    s = base.with_params(p_continue=0.0)
    S = S0.copy()
    for t in range(1, 15):
        nxt, _, _, _ = oracle_lib.step(s, t, S)
        assert np.all(nxt[S == 1] == 2)
        S = nxt
    # p_continue = 1: nothing ever burns out
    r = oracle_lib.run(base.with_params(p_continue=1.0), 15)
    assert (r["S"] == 2).sum() == 0 and (r["S"] == 1).sum() > 1


# ----------------------------------------------------------------- Eq. 10

def test_bce_crop_closed_form(oracle_lib):
    yhat = np.zeros((4, 4))
    y = np.zeros((4, 4), np.uint8)
    yhat[1, 1] = 0.5
    y[2, 3] = 1
    L, lam = oracle_lib.loss(yhat, y, 0)
    want = (math.log1p(math.exp(0.5)) + 5 * math.log(2.0)) / 6.0
    assert L == pytest.approx(want, rel=1e-14)
    assert lam[0, 0] == 0.0 and lam[3, 0] == 0.0
    assert lam[2, 3] == pytest.approx((0.5 - 1.0) / 6.0, rel=1e-14)
    L0, _ = oracle_lib.loss(np.zeros((4, 4)), np.zeros((4, 4), np.uint8), 0)
    assert L0 == 0.0


def test_mse_pool_closed_form(oracle_lib):
    y = np.zeros((8, 8), np.uint8)
    y[:4, :4] = 1
    yhat = y.astype(np.float64).copy()
    yhat[5, 6] = 0.8
    L, _ = oracle_lib.loss(yhat, y, 2)
    assert L == pytest.approx((0.8 / 16) ** 2 / 4, rel=1e-14)


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_loss_lambda_by_finite_differences(oracle_lib, kind):
    rng = np.random.default_rng(kind)
    yhat = np.where(rng.random((9, 10)) < 0.4, rng.random((9, 10)), 0.0)
    yhat[0, :] = 0.0
    y = (rng.random((9, 10)) < 0.3).astype(np.uint8)
    y[0, :] = 0
    L, lam = oracle_lib.loss(yhat, y, kind)
    h = 1e-6
    for (r, c) in [(1, 1), (4, 5), (8, 9), (3, 0)]:
        if yhat[r, c] == 0.0 and y[r, c] == 0 and kind != 2:
            continue  # moving a zero cell can change the crop
        yp, ym = yhat.copy(), yhat.copy()
        yp[r, c] += h
        ym[r, c] -= h
        fd = (oracle_lib.loss(yp, y, kind)[0] - oracle_lib.loss(ym, y, kind)[0]) / (2 * h)
        assert lam[r, c] == pytest.approx(fd, rel=1e-6, abs=1e-10)


# --------------------------------------------------------------- gradient

def _calib_problem(oracle_lib, H=32, W=32, T=24):
    s = synth.make_lakes(H, W, 21, T=T, n_ignitions=2)
    s.seed = 77
    target = oracle_lib.run(s.with_params(0.7, 0.05, 0.06, 0.1), T)["S"]
    y = (target != 0).astype(np.uint8)
    return s, y


def test_gradient_matches_crn_finite_differences(oracle_lib):
    s, y = _calib_problem(oracle_lib)
    r = oracle_lib.run(s, s.T, want_yhat=True)
    L, lam = oracle_lib.loss(r["yhat"], y, 1)
    g = oracle_lib.grad(s, s.T, lam)
    fd, flips = oracle_lib.fd_grad(s, s.T, y, kind=1)
    assert np.all(flips == 0), flips
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-12)
    assert np.all(np.abs(g) > 0)


def test_gradient_vanishing_cases(oracle_lib):
    # flat terrain: dL/da = 0; calm: dL/dc1 = dL/dc2 = 0
    s = synth.make_plain(20, 20, 5, e_max=0.0, wind_speed=0.0)
    r = oracle_lib.run(s, 12, want_yhat=True)
    y = (oracle_lib.run(s.with_params(p_h=0.8), 12)["S"] != 0).astype(np.uint8)
    _, lam = oracle_lib.loss(r["yhat"], y, 0)
    g = oracle_lib.grad(s, 12, lam)
    assert g[1] == 0.0 and g[2] == 0.0 and g[3] == 0.0
    assert g[0] != 0.0


# ------------------------------------------ slope tensor input, Eq. 11-12

def test_slope_tensor_layout_and_equivalence(oracle_lib):
    """The paper-layout slope tensor puts Eq. 1's angle of the edge
    (r+dr, c+dc) -> (r, c) at [r][c][dr+1][dc+1]; feeding it back reproduces
    the elevation-based p_ignite (up to the FP32 rounding of the angles)."""
    s = flat_scenario(3, 3)
    E = np.zeros((3, 3), np.float32)
    E[1, 1] = 30.0                      # the centre is l metres above the west cell
    s.elevation = E
    t = oracle_lib.slope_tensor(s)
    assert t[1, 1, 1, 0] == pytest.approx(45.0, abs=1e-5)
    assert t[1, 1, 1, 1] == 0.0
    assert t[1, 0, 1, 2] == pytest.approx(-45.0, abs=1e-5)   # west cell, from the centre
    assert t[0, 0, 0, 0] == 0.0                               # out-of-grid slot
    s2, S = random_small(17, 23, 31, per_cell_wind=True)
    ref = oracle_lib.pignite_map(s2, S)
    s3 = dataclasses.replace(s2)
    s3.slope_deg = oracle_lib.slope_tensor(s2)
    s3.elevation = None
    got = oracle_lib.pignite_map(s3, S)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-12)


def test_jaccard_and_manhattan_closed_forms(oracle_lib):
    A = np.zeros((4, 4), bool)
    B = np.zeros((4, 4), bool)
    A[:2, :2] = True
    B[1:3, 1:3] = True
    assert oracle_lib.jaccard(A, A) == 1.0
    assert oracle_lib.jaccard(A, ~A) == 0.0
    assert oracle_lib.jaccard(A, B) == pytest.approx(1 / 7)
    assert oracle_lib.manhattan([1, 5, 9], [2, 5, 7]) == 3.0
    assert oracle_lib.manhattan([3, 3], [3, 3]) == 0.0


def test_next_cells_is_the_rule_of_step(oracle_lib):
    """The per-cell rule used for sampled checks on very large grids is the
    rule of the whole-grid step."""
    s, S = random_small(23, 31, 41, per_cell_wind=True)
    full, tie, pmap, _ = oracle_lib.step(s, 9, S, tie_eps=1e-3)
    rr, cc = np.divmod(np.arange(s.H * s.W), s.W)
    nxt, p, t = oracle_lib.next_cells(s, 9, S, rr, cc, tie_eps=1e-3)
    assert np.array_equal(nxt.reshape(S.shape), full)
    assert np.array_equal(t.reshape(S.shape), tie.astype(bool))
    np.testing.assert_array_equal(p.reshape(S.shape), pmap)


# ------------------------------------------------------ near ties, threads

def test_near_tie_needs_a_trial_that_rounding_can_change(oracle_lib):
    """An ignition trial is a near tie when |u - p_ignite| <= eps; at a cell
    without fuel (or with p_h = 0) every edge has x = 0 (Eq. 2), p_ignite is
    exactly 0 in any precision and the trial is never a tie, whatever eps."""
    eps = 0.5   # wide window, so that ordinary draws qualify
    base = flat_scenario(3, 3)
    S = np.zeros((3, 3), np.uint8)
    S[0, 1] = 1                          # one burning neighbour of the centre
    pb = oracle_lib.Problem(base)
    t = next(t for t in range(1, 1000) if oracle_lib.draws(pb, t, 4)[0] <= 0.45)
    u = oracle_lib.draws(pb, t, 4)[0]
    # fuelled centre: p = tanh(c p_h) ~ 0.58 lies within eps of u
    nxt, p, tie = oracle_lib.next_cells(base, t, S, [1], [1], tie_eps=eps)
    assert p[0] == pytest.approx(math.tanh(C * float(np.float32(0.58))), rel=1e-12)
    assert tie[0] == (abs(u - p[0]) <= eps) and tie[0]
    # no fuel at the centre: p = 0, |u - p| <= eps, still not a tie
    nofuel = dataclasses.replace(base, p_veg=base.p_veg.copy())
    nofuel.p_veg[1, 1] = -1.0
    nxt, p, tie = oracle_lib.next_cells(nofuel, t, S, [1], [1], tie_eps=eps)
    assert p[0] == 0.0 and nxt[0] == 0 and not tie[0]
    # p_h = 0: same
    nxt, p, tie = oracle_lib.next_cells(base.with_params(p_h=0.0), t, S, [1], [1], tie_eps=eps)
    assert p[0] == 0.0 and nxt[0] == 0 and not tie[0]


def random_lakes_case(seed):
    return synth.make_lakes(70, 83, seed, T=40, n_ignitions=3)


def test_threaded_build_equals_plain_build(oracle_lib):
    """The OpenMP build splits rows over threads; results must not change."""
    s = random_lakes_case(5)
    try:
        oracle_lib.set_threads(1)
        a = oracle_lib.run(s, 40, want_yhat=True, want_tstep=True)
        pa = oracle_lib.pignite_map(s, a["S"])
        oracle_lib.set_threads(4)
        b = oracle_lib.run(s, 40, want_yhat=True, want_tstep=True)
        pbm = oracle_lib.pignite_map(s, b["S"])
    finally:
        oracle_lib.set_threads(1)
    assert np.array_equal(a["S"], b["S"]) and a["ties"] == b["ties"]
    assert np.array_equal(a["yhat"], b["yhat"]) and np.array_equal(a["tstep"], b["tstep"])
    assert np.array_equal(pa, pbm)


def test_run_ties_lists_the_ties_of_each_step(oracle_lib):
    s = random_lakes_case(6)
    eps = 2e-3   # wide enough that a short run has ties to list
    r = oracle_lib.run_ties(s, 40, tie_eps=eps)
    S = oracle_lib.initial_state(s)
    want = []
    for t in range(1, 41):
        S, tie, _, _ = oracle_lib.step(s, t, S, tie_eps=eps)
        want += [(t, int(c)) for c in np.flatnonzero(tie.ravel())]
    assert len(want) > 5 and r["ties"] == len(want)
    assert list(zip(r["tie_step"].tolist(), r["tie_cell"].tolist())) == want
    assert np.array_equal(r["S"], S)


# ------------------------------------------------------------ Algorithm 1

def test_adamw_matches_torch_cpu(oracle_lib):
    """The oracle's AdamW (decoupled weight decay) reproduces torch's CPU
    AdamW in FP64 step for step, with the paper's lr and torch's defaults."""
    import torch
    rng = np.random.default_rng(3)
    th0 = rng.uniform(0.1, 0.9, 4)
    ref = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([ref], lr=5e-3)
    mine = oracle_lib.AdamW(th0, lr=5e-3)
    for _ in range(12):
        g = rng.standard_normal(4) * rng.uniform(1e-3, 10.0)
        ref.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        mine.step(g)
        np.testing.assert_allclose(mine.theta, ref.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_algorithm1_sequence_clamps_and_metrics(oracle_lib):
    """Oracle Algorithm 1: parameters stay in the clamp box, the first
    iteration's gradient is the analytic gradient at theta0, Jaccard equals
    1 and Manhattan 0 when the observations are the run's own states."""
    s = synth.make_lakes(48, 40, 71, T=30, n_ignitions=2)
    th0 = [0.58, 0.078, 0.045, 0.131]
    base = s.with_params(*th0)
    obs = [(oracle_lib.run(dataclasses.replace(base, seed=1000), 10 * (k + 1))["S"] != 0)
           .astype(np.uint8).ravel() for k in range(3)]
    hist = oracle_lib.calibrate_sequence(s, obs, th0, interval=10, epochs=1, lr=1e-2)
    assert [h["iteration"] for h in hist] == [0, 1, 2]
    r0 = oracle_lib.run(dataclasses.replace(base, seed=1000), 10, want_yhat=True)
    L, lam = oracle_lib.loss(r0["yhat"], obs[0].reshape(s.H, s.W), 0)
    assert hist[0]["loss"] == L
    np.testing.assert_array_equal(hist[0]["grad"],
                                  oracle_lib.grad(dataclasses.replace(base, seed=1000), 10, lam))
    assert hist[0]["jaccard"] == 1.0 and hist[0]["manhattan"] == 0
    for h in hist:
        assert np.all(h["theta"] >= oracle_lib.CLAMP_LO) and np.all(h["theta"] <= oracle_lib.CLAMP_HI)
