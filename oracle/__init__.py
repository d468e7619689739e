"""Python handle on the FP64 CPU oracle (``fireoracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the benchmark's CPU-baseline leg, never by the product package.  It
shares no code with the GPU path; both only consume the arrays produced by
the ``synth`` generators.

Scenario objects are duck-typed: anything with ``H, W, cell_m, seed,
scenario_id, p_veg, p_den, elevation, wind_speed, wind_dir,
wind_speed_scalar, wind_dir_scalar, init_burning`` and the parameters
``p_h, a, c1, c2, p_continue`` works.  FP32 inputs and FP32 parameter values
are widened to double before any arithmetic.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# The same source built with OpenMP: fo_step and fo_pignite_map split their
# row loops over threads (the per-cell arithmetic is unchanged).
_LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_libs = {}
_threads = 1

# FP32 rounding of the f_p constant 1.1486328125 (Eq. 5 / 8).
C_F32 = float(np.float32(1.1486328125))


def build(force: bool = True) -> str:
    """Compile ``fireoracle.c`` into ``liboracle.so`` (gcc, FP64, no fast-math)
    and, from the same source with OpenMP, ``liboracle_omp.so``."""
    src = os.path.join(_HERE, "fireoracle.c")
    for path, extra in ((_LIB_PATH, []), (_LIB_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                                   "-ffp-contract=off"] + extra + ["-o", tmp, src, "-lm"])
            os.replace(tmp, path)
    return _LIB_PATH


def set_threads(n: int) -> int:
    """Use n host threads for the row loops of step / run / p_ignite maps
    (n <= 1: the plain single-threaded build).  Returns the count in use."""
    global _threads
    _threads = max(1, int(n))
    lib = _load()
    return int(lib.fo_threads(_threads if _threads > 1 else 0))


def threads() -> int:
    return _threads


class _Problem(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_int32), ("W", ctypes.c_int32),
        ("cell_m", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("scenario", ctypes.c_uint32),
        ("p_h", ctypes.c_double), ("a", ctypes.c_double),
        ("c1", ctypes.c_double), ("c2", ctypes.c_double),
        ("p_continue", ctypes.c_double),
        ("c", ctypes.c_double),
        ("p_veg", ctypes.c_void_p), ("p_den", ctypes.c_void_p), ("elev", ctypes.c_void_p),
        ("wind_speed", ctypes.c_void_p), ("wind_dir", ctypes.c_void_p),
        ("wind_speed_scalar", ctypes.c_double), ("wind_dir_scalar", ctypes.c_double),
        ("slope9", ctypes.c_void_p),
    ]


def _load():
    key = "omp" if _threads > 1 else "plain"
    if key in _libs:
        return _libs[key]
    path = _LIB_OMP_PATH if key == "omp" else _LIB_PATH
    if not os.path.exists(path):
        build(force=False)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(_Problem)
    vp = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.fo_philox4x32_10.argtypes = [vp, vp, vp]
    lib.fo_draws.argtypes = [P, i32, i64, vp, vp]
    lib.fo_edge_q.argtypes = [P, i32, i32, i32, i32, vp, vp]
    lib.fo_edge_q.restype = dbl
    lib.fo_pignite_cell.argtypes = [P, vp, i32, i32]
    lib.fo_pignite_cell.restype = dbl
    lib.fo_pignite_map.argtypes = [P, vp, vp]
    lib.fo_dpignite_cell.argtypes = [P, vp, i32, i32, vp]
    lib.fo_step.argtypes = [P, i32, vp, vp, vp, vp, dbl, vp]
    lib.fo_step.restype = i64
    lib.fo_next_cell.argtypes = [P, i32, vp, i32, i32, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int), dbl]
    lib.fo_next_cell.restype = ctypes.c_uint8
    lib.fo_run.argtypes = [P, i32, i32, vp, vp, vp, dbl]
    lib.fo_run.restype = i64
    lib.fo_run_ties.argtypes = [P, i32, i32, vp, vp, vp, dbl, vp, vp, i64]
    lib.fo_run_ties.restype = i64
    lib.fo_threads.argtypes = [ctypes.c_int]
    lib.fo_threads.restype = ctypes.c_int
    lib.fo_loss.argtypes = [i32, i32, vp, vp, i32, vp]
    lib.fo_loss.restype = dbl
    lib.fo_grad.argtypes = [P, i32, vp, vp, vp]
    lib.fo_slope_tensor.argtypes = [P, vp]
    if key == "omp":
        lib.fo_threads(_threads)
    _libs[key] = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class Problem:
    """A scenario frozen into the oracle's C struct (keeps its arrays alive)."""

    def __init__(self, scn, c=C_F32, **override):
        self.H, self.W = int(scn.H), int(scn.W)
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
        self.p_veg, self.p_den = f(scn.p_veg), f(scn.p_den)
        self.elev = f(scn.elevation)
        self.ws, self.wd = f(scn.wind_speed), f(scn.wind_dir)
        self.slope9 = f(getattr(scn, "slope_deg", None))
        par = {k: float(np.float32(getattr(scn, k)))
               for k in ("p_h", "a", "c1", "c2", "p_continue")}
        par.update({k: float(v) for k, v in override.items()
                    if k in ("p_h", "a", "c1", "c2", "p_continue")})
        self.params = par
        self.seed = int(override.get("seed", scn.seed))
        self.scenario = int(override.get("scenario_id", scn.scenario_id))
        self.s = _Problem(self.H, self.W, float(scn.cell_m), self.seed, self.scenario,
                          par["p_h"], par["a"], par["c1"], par["c2"], par["p_continue"],
                          float(c), _ptr(self.p_veg), _ptr(self.p_den), _ptr(self.elev),
                          _ptr(self.ws), _ptr(self.wd),
                          float(np.float32(scn.wind_speed_scalar)),
                          float(np.float32(scn.wind_dir_scalar)), _ptr(self.slope9))
        self.init_burning = np.ascontiguousarray(scn.init_burning, dtype=np.uint8)

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _problem(scn, **kw):
    return scn if isinstance(scn, Problem) else Problem(scn, **kw)


def philox4x32_10(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.fo_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def draws(scn, t, cell):
    lib = _load()
    pb = _problem(scn)
    ui, uc = ctypes.c_double(), ctypes.c_double()
    lib.fo_draws(pb.ref, int(t), int(cell), ctypes.byref(ui), ctypes.byref(uc))
    return ui.value, uc.value


def edge_q(scn, r, c, dr, dc, **kw):
    """(q, theta_s in degrees, cos(delta)) of the edge (r+dr, c+dc) -> (r, c)."""
    lib = _load()
    pb = _problem(scn, **kw)
    th, cd = ctypes.c_double(), ctypes.c_double()
    q = lib.fo_edge_q(pb.ref, r, c, dr, dc, ctypes.byref(th), ctypes.byref(cd))
    return q, th.value, cd.value


def slope_tensor(scn):
    """Eq. 1 in the paper's H x W x 3 x 3 layout (degrees, FP32)."""
    lib = _load()
    pb = _problem(scn)
    out = np.zeros((pb.H, pb.W, 3, 3), dtype=np.float32)
    lib.fo_slope_tensor(pb.ref, out.ctypes.data)
    return out


def affected(S):
    """Burning or burned cells of a state (the affected area of Eq. 11-12)."""
    return np.asarray(S) != 0


def jaccard(A, B):
    """Eq. 11: |A intersect B| / |A union B| of two affected-area masks."""
    A, B = np.asarray(A, bool), np.asarray(B, bool)
    u = np.count_nonzero(A | B)
    return 1.0 if u == 0 else np.count_nonzero(A & B) / u


def manhattan(counts_a, counts_b):
    """Eq. 12: sum over time of |A_t - B_t| of affected-cell counts."""
    return float(np.sum(np.abs(np.asarray(counts_a, float) - np.asarray(counts_b, float))))


def initial_state(scn):
    return (np.asarray(scn.init_burning) != 0).astype(np.uint8)


def pignite_map(scn, S, **kw):
    lib = _load()
    pb = _problem(scn, **kw)
    S = np.ascontiguousarray(S, dtype=np.uint8)
    out = np.zeros((pb.H, pb.W), dtype=np.float64)
    lib.fo_pignite_map(pb.ref, S.ctypes.data, out.ctypes.data)
    return out


def pignite_cell(scn, S, r, c, **kw):
    lib = _load()
    pb = _problem(scn, **kw)
    S = np.ascontiguousarray(S, dtype=np.uint8)
    return lib.fo_pignite_cell(pb.ref, S.ctypes.data, r, c)


def dpignite_cell(scn, S, r, c, **kw):
    lib = _load()
    pb = _problem(scn, **kw)
    S = np.ascontiguousarray(S, dtype=np.uint8)
    g = np.zeros(4, dtype=np.float64)
    lib.fo_dpignite_cell(pb.ref, S.ctypes.data, r, c, g.ctypes.data)
    return g


def next_cells(scn, t, S_prev, rows, cols, tie_eps=1e-5, **kw):
    """The per-cell rule of `step` at the listed cells only (for grids too
    large to step whole): returns (next state, p_ignite, tie flag) arrays."""
    lib = _load()
    pb = _problem(scn, **kw)
    S_prev = np.ascontiguousarray(S_prev, dtype=np.uint8)
    n = len(rows)
    nxt = np.zeros(n, np.uint8)
    pv = np.zeros(n, np.float64)
    tv = np.zeros(n, bool)
    p = ctypes.c_double()
    tie = ctypes.c_int()
    for k in range(n):
        nxt[k] = lib.fo_next_cell(pb.ref, int(t), S_prev.ctypes.data, int(rows[k]), int(cols[k]),
                                  ctypes.byref(p), ctypes.byref(tie), float(tie_eps))
        pv[k] = p.value
        tv[k] = bool(tie.value)
    return nxt, pv, tv


def step(scn, t, S_prev, tie_eps=1e-5, yhat=None, **kw):
    """One step: returns (S_next, tie mask, p_ignite map of S_prev, tie count)."""
    lib = _load()
    pb = _problem(scn, **kw)
    S_prev = np.ascontiguousarray(S_prev, dtype=np.uint8)
    nxt = np.zeros_like(S_prev)
    tie = np.zeros_like(S_prev)
    pmap = np.zeros(S_prev.shape, dtype=np.float64)
    n = lib.fo_step(pb.ref, int(t), S_prev.ctypes.data, nxt.ctypes.data, _ptr(yhat),
                    tie.ctypes.data, float(tie_eps), pmap.ctypes.data)
    return nxt, tie.astype(bool), pmap, int(n)


def run(scn, T, t0=0, S=None, tie_eps=1e-5, want_yhat=False, want_tstep=False, **kw):
    """Steps t0+1..t0+T from S (default: the ignition state).

    Returns dict(S=final state, ties=count, yhat=..., tstep=...).
    ``yhat`` starts at 1 on initially burning cells (their accumulator value
    is a constant) and 0 elsewhere; ``tstep`` is the ignition step (0 for
    the initial cells, -1 for cells never ignited).
    """
    lib = _load()
    pb = _problem(scn, **kw)
    S = initial_state(scn) if S is None else np.array(S, dtype=np.uint8, copy=True)
    S = np.ascontiguousarray(S)
    yhat = None
    if want_yhat:
        yhat = (S == 1).astype(np.float64)
    tstep = None
    if want_tstep:
        tstep = np.where(S == 1, 0, -1).astype(np.int32)
    ties = lib.fo_run(pb.ref, int(t0), int(T), S.ctypes.data, _ptr(yhat), _ptr(tstep),
                      float(tie_eps))
    return {"S": S, "ties": int(ties), "yhat": yhat, "tstep": tstep}


def run_ties(scn, T, t0=0, S=None, tie_eps=1e-5, cap=1 << 20, want_yhat=False, **kw):
    """Like ``run``, and lists the near ties: returns dict(S=..., ties=count,
    tie_step=int32 array, tie_cell=int64 array (r*W + c), yhat=...), ties in
    step and cell order."""
    lib = _load()
    pb = _problem(scn, **kw)
    S = initial_state(scn) if S is None else np.array(S, dtype=np.uint8, copy=True)
    S = np.ascontiguousarray(S)
    yhat = (S == 1).astype(np.float64) if want_yhat else None
    ts = np.zeros(cap, np.int32)
    tc = np.zeros(cap, np.int64)
    n = lib.fo_run_ties(pb.ref, int(t0), int(T), S.ctypes.data, _ptr(yhat), None,
                        float(tie_eps), ts.ctypes.data, tc.ctypes.data, int(cap))
    m = min(int(n), cap)
    return {"S": S, "ties": int(n), "tie_step": ts[:m].copy(), "tie_cell": tc[:m].copy(),
            "yhat": yhat}


def loss(yhat, y, kind=0):
    """Eq. 10 reading: returns (loss, dL/dyhat)."""
    lib = _load()
    yhat = np.ascontiguousarray(yhat, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    H, W = yhat.shape
    lam = np.zeros_like(yhat)
    L = lib.fo_loss(H, W, yhat.ctypes.data, y.ctypes.data, int(kind), lam.ctypes.data)
    return L, lam


def grad(scn, T, lam, **kw):
    """Analytic gradient of sum(lam * yhat) w.r.t. (p_h, a, c1, c2)."""
    lib = _load()
    pb = _problem(scn, **kw)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    g = np.zeros(4, dtype=np.float64)
    lib.fo_grad(pb.ref, int(T), pb.init_burning.ctypes.data, lam.ctypes.data,
                g.ctypes.data)
    return g


PARAM_NAMES = ("p_h", "a", "c1", "c2")


def fd_grad(scn, T, y, kind=0, h_rel=1e-7, h_min=1e-9):
    """Central finite differences of L(yhat(theta)) with common random numbers.

    Returns (g, flips): flips[k] counts cells whose ignition step differs
    between the +h and -h runs for parameter k (0 means the discrete
    trajectory was identical and the difference quotient is exact up to
    O(h^2) and rounding).
    """
    base = {k: float(np.float32(getattr(scn, k))) for k in PARAM_NAMES}
    g = np.zeros(4)
    flips = np.zeros(4, dtype=np.int64)
    for k, name in enumerate(PARAM_NAMES):
        h = max(abs(base[name]) * h_rel, h_min)
        outs = []
        for sgn in (+1, -1):
            ov = dict(base)
            ov[name] = base[name] + sgn * h
            r = run(scn, T, want_yhat=True, want_tstep=True, **ov)
            outs.append(r)
        Lp = loss(outs[0]["yhat"], y, kind)[0]
        Lm = loss(outs[1]["yhat"], y, kind)[0]
        g[k] = (Lp - Lm) / (2 * h)
        flips[k] = int(np.count_nonzero(outs[0]["tstep"] != outs[1]["tstep"]))
    return g, flips


# ----------------------------------------------------------- Algorithm 1

# Clamp ranges of Algorithm 1: p_h in [0.2, 1]; a, c1, c2 in [0, 1].
CLAMP_LO = np.array([0.2, 0.0, 0.0, 0.0])
CLAMP_HI = np.array([1.0, 1.0, 1.0, 1.0])


class AdamW:
    """AdamW (Adam with decoupled weight decay, Loshchilov & Hutter, ICLR 2019)
    in FP64, with the defaults the paper's optimiser uses (Sec. 2.3: lr 5e-3;
    betas (0.9, 0.999), eps 1e-8, weight decay 0.01):
        theta <- theta (1 - lr wd)
        m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2
        theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, theta, lr=5e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01):
        self.theta = np.array(theta, dtype=np.float64)
        self.lr, self.b1, self.b2 = float(lr), float(betas[0]), float(betas[1])
        self.eps, self.wd = float(eps), float(weight_decay)
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0

    def step(self, g):
        g = np.asarray(g, dtype=np.float64)
        self.t += 1
        self.theta = self.theta * (1.0 - self.lr * self.wd)
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        self.theta = self.theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)
        return self.theta


def calibrate_sequence(scn, observations, theta0, interval, epochs=1, lr=5e-3, kind=0,
                       winds=None, seed0=1000):
    """Algorithm 1 with several observations per epoch, for one scenario: in
    epoch ep the seed is seed0 + ep for every iteration; iteration it replays
    the fire from its start for (it + 1) * interval steps under the current
    parameters (rounded to FP32, the working precision) and, if given, the
    wind winds[it] = (speed field or None, direction field or None, speed
    scalar, direction scalar); takes the Eq. 10 loss against
    observations[it] and its gradient, one AdamW step and the clamps.
    Per iteration it also reports Eq. 11 (Jaccard of the affected areas at
    the observation time) and Eq. 12 (the running sum over the epoch's
    observation times of |affected count - observed count|).
    Returns a list of dicts (epoch, iteration, loss, grad, theta, jaccard,
    manhattan)."""
    import dataclasses
    opt = AdamW(theta0, lr=lr)
    out = []
    for ep in range(epochs):
        manhattan = 0
        for it, obs in enumerate(observations):
            th = [float(np.float32(x)) for x in opt.theta]
            sc = dataclasses.replace(scn, seed=seed0 + ep)
            sc = sc.with_params(th[0], th[1], th[2], th[3])
            if winds is not None:
                ws, wd, ws0, wd0 = winds[it]
                sc = dataclasses.replace(sc, wind_speed=ws, wind_dir=wd,
                                         wind_speed_scalar=ws0, wind_dir_scalar=wd0)
            T = (it + 1) * int(interval)
            y = np.asarray(obs, dtype=np.uint8).reshape(scn.H, scn.W)
            r = run(sc, T, want_yhat=True)
            L, lam = loss(r["yhat"], y, kind)
            g = grad(sc, T, lam)
            A = affected(r["S"])
            manhattan += abs(int(np.count_nonzero(A)) - int(np.count_nonzero(y)))
            opt.step(g)
            opt.theta = np.minimum(np.maximum(opt.theta, CLAMP_LO), CLAMP_HI)
            out.append({"epoch": ep, "iteration": it, "loss": L, "grad": g,
                        "theta": opt.theta.copy(), "jaccard": jaccard(A, y != 0),
                        "manhattan": manhattan, "S": r["S"]})
    return out
