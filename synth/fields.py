"""Synthetic landscapes standing in for the paper's LANDFIRE / ERA5 rasters.

The paper calibrates on real Californian ecoregions (30 m cells, Appendix A,
"Dataset"); those rasters are not available here, so every workload is drawn
from ``numpy.random.default_rng(seed)`` with a fixed draw order:

1. vegetation class, 2. density class, 3. non-burnable mask, 4. elevation
noise, 5. wind-speed noise, 6. wind-direction noise, 7. ignition positions.

Smoothing is a Gaussian applied in the Fourier domain (periodic boundary;
``scipy.ndimage.fourier_gaussian`` on a real FFT), smoothed fields are
min-max scaled, non-burnable cells get ``p_veg = -1`` (the paper's
"very small p_veg" reading of the no-fuel state, Sec. 2.2), and ignition cells
are forced burnable.  Grid orientation: row 0 is north, rows run south,
columns run east.  Wind direction is the heading the wind blows toward, in
degrees counter-clockwise from east (Sec. 2.1, wind inputs).

Nothing here computes a propagation probability or a state transition.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.fft
from scipy.ndimage import fourier_gaussian, gaussian_filter

# Vegetation and density class -> scaling factor (the workload definitions).
VEG_CLASSES = np.array([-0.3, 0.0, 0.4, 0.2], dtype=np.float32)
DEN_CLASSES = np.array([-0.4, 0.0, 0.3], dtype=np.float32)

# (p_h, a, c1, c2) used to generate calibration targets, and the paper-style
# default parameter set; p_continue = 0.3.
PARAMS_TRUE = (0.58, 0.078, 0.045, 0.131)
P_CONTINUE = 0.3

# Normaliser constant of Eq. 5/8, stored as the FP32 value both sides use.
C_NORMALISER = float(np.float32(1.1486328125))

CELL_M = 30.0


@dataclasses.dataclass
class Scenario:
    """One fire scenario: fields, parameters, ignition and horizon.

    All arrays are C-contiguous FP32 (fields) or uint8 (ignition), row-major
    H x W.  ``wind_speed`` / ``wind_dir`` are None for spatially uniform wind,
    in which case the scalars apply.
    """

    H: int
    W: int
    p_veg: np.ndarray
    p_den: np.ndarray
    elevation: np.ndarray
    wind_speed: Optional[np.ndarray]
    wind_dir: Optional[np.ndarray]
    wind_speed_scalar: float
    wind_dir_scalar: float
    init_burning: np.ndarray
    p_h: float = PARAMS_TRUE[0]
    a: float = PARAMS_TRUE[1]
    c1: float = PARAMS_TRUE[2]
    c2: float = PARAMS_TRUE[3]
    p_continue: float = P_CONTINUE
    cell_m: float = CELL_M
    seed: int = 0
    scenario_id: int = 0
    T: int = 100
    # Optional per-edge slope angles in degrees, H x W x 3 x 3 (the paper's
    # slope tensor layout); when given it replaces the elevation-based Eq. 1.
    slope_deg: Optional[np.ndarray] = None

    @property
    def params(self):
        """(p_h, a, c1, c2, p_continue) rounded to FP32."""
        return tuple(float(np.float32(v)) for v in
                     (self.p_h, self.a, self.c1, self.c2, self.p_continue))

    def with_params(self, p_h=None, a=None, c1=None, c2=None, p_continue=None):
        d = dataclasses.replace(self)
        for k, v in (("p_h", p_h), ("a", a), ("c1", c1), ("c2", c2),
                     ("p_continue", p_continue)):
            if v is not None:
                setattr(d, k, float(np.float32(v)))
        return d


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def _minmax(x, lo, hi):
    mn, mx = float(x.min()), float(x.max())
    if mx > mn:
        x = (x - mn) / (mx - mn)
    else:
        x = np.zeros_like(x)
    return lo + (hi - lo) * x


def _smooth(rng, H, W, sigma):
    x = rng.standard_normal((H, W))
    f = fourier_gaussian(scipy.fft.rfft2(x, workers=-1), sigma=sigma, n=W)
    return scipy.fft.irfft2(f, s=(H, W), workers=-1)


def _base(rng, H, W, nonburn, nonburn_frac, e_sigma, e_max):
    veg = VEG_CLASSES[rng.integers(0, 4, size=(H, W))]
    den = DEN_CLASSES[rng.integers(0, 3, size=(H, W))]
    if nonburn == "iid":
        mask = rng.random((H, W)) < nonburn_frac
    elif nonburn == "lakes":
        f = _smooth(rng, H, W, 8.0)
        mask = f > np.quantile(f, 1.0 - nonburn_frac)
    else:
        mask = np.zeros((H, W), dtype=bool)
    veg = np.where(mask, np.float32(-1.0), veg)
    elev = _minmax(_smooth(rng, H, W, e_sigma), 0.0, e_max)
    return veg, den, elev


def _ignite(veg, cells):
    ign = np.zeros(veg.shape, dtype=np.uint8)
    for (r, c) in cells:
        ign[r, c] = 1
        if veg[r, c] <= -1.0:
            veg[r, c] = 0.0  # forced burnable
    return ign


def make_rough(H, W, seed, *, nonburn_frac=0.05, e_max=5.0, T=100):
    """Unsmoothed fields for very large grids (index and edge tests at the
    paper's largest side): iid classes and non-burnable cells, iid elevation in
    [0, e_max] m, iid per-cell wind (0-12 m/s, [0, 360) degrees).  Generated
    in float32 draws so that a 14 000 x 14 000 grid takes seconds."""
    rng = np.random.default_rng(seed)
    veg = VEG_CLASSES[rng.integers(0, 4, size=(H, W), dtype=np.int8)]
    den = DEN_CLASSES[rng.integers(0, 3, size=(H, W), dtype=np.int8)]
    veg = np.where(rng.random((H, W), dtype=np.float32) < nonburn_frac, np.float32(-1.0), veg)
    elev = rng.random((H, W), dtype=np.float32) * np.float32(e_max)
    ws = rng.random((H, W), dtype=np.float32) * np.float32(12.0)
    wd = rng.random((H, W), dtype=np.float32) * np.float32(360.0)
    ign = np.zeros((H, W), dtype=np.uint8)
    s = Scenario(H=H, W=W, p_veg=_f32(veg), p_den=_f32(den), elevation=_f32(elev),
                 wind_speed=_f32(ws), wind_dir=_f32(wd),
                 wind_speed_scalar=0.0, wind_dir_scalar=0.0,
                 init_burning=ign, seed=seed, scenario_id=0, T=T)
    return s.with_params(*s.params)


def make_plain(H, W, seed, *, nonburn_frac=0.05, e_sigma=8.0, e_max=300.0,
               wind_speed=5.0, wind_dir=45.0, ignitions=None, T=100,
               scenario_id=0, params=None):
    """Config-0 style landscape: iid non-burnable cells, uniform wind."""
    rng = np.random.default_rng(seed)
    veg, den, elev = _base(rng, H, W, "iid", nonburn_frac, e_sigma, e_max)
    if ignitions is None:
        ignitions = [(H // 2, W // 2)]
    ign = _ignite(veg, ignitions)
    s = Scenario(H=H, W=W, p_veg=_f32(veg), p_den=_f32(den), elevation=_f32(elev),
                 wind_speed=None, wind_dir=None,
                 wind_speed_scalar=float(np.float32(wind_speed)),
                 wind_dir_scalar=float(np.float32(wind_dir)),
                 init_burning=ign, seed=seed, scenario_id=scenario_id, T=T)
    if params is not None:
        s = s.with_params(*params)
    return s.with_params(*s.params)


def make_lakes(H, W, seed, *, nonburn_frac=0.10, e_sigma=8.0, e_max=300.0,
               n_ignitions=5, ignition_patch=None, T=500, scenario_id=0,
               params=None):
    """Config-1 style landscape: lakes, per-cell smooth wind, random ignitions."""
    rng = np.random.default_rng(seed)
    veg, den, elev = _base(rng, H, W, "lakes", nonburn_frac, e_sigma, e_max)
    ws = _minmax(_smooth(rng, H, W, 32.0), 0.0, 12.0)
    wd = np.mod(_minmax(_smooth(rng, H, W, 32.0), 0.0, 360.0), 360.0)
    if ignition_patch is not None:
        r0, c0, n = ignition_patch
        cells = [(r, c) for r in range(r0, r0 + n) for c in range(c0, c0 + n)]
    else:
        rr = rng.integers(0, H, size=n_ignitions)
        cc = rng.integers(0, W, size=n_ignitions)
        cells = list(zip(rr.tolist(), cc.tolist()))
    ign = _ignite(veg, cells)
    s = Scenario(H=H, W=W, p_veg=_f32(veg), p_den=_f32(den), elevation=_f32(elev),
                 wind_speed=_f32(ws), wind_dir=_f32(wd),
                 wind_speed_scalar=0.0, wind_dir_scalar=0.0,
                 init_burning=ign, seed=seed, scenario_id=scenario_id, T=T)
    if params is not None:
        s = s.with_params(*params)
    return s.with_params(*s.params)


def config0(seed=0):
    """128 x 128, 5 % iid non-burnable, uniform wind 5 m/s toward 45 deg, T = 100."""
    return make_plain(128, 128, seed, T=100)


def config1(seed=1, size=1024, T=500):
    """1024 x 1024 with 10 % lakes, per-cell wind, 5 random ignitions, T = 500."""
    return make_lakes(size, size, seed, T=T)


def config2(seed=2, size=4096, T=1000):
    """4096 x 4096, elevation 0-1500 m (sigma 32), 20 x 20 central patch, T = 1000."""
    n = 20
    r0 = size // 2 - n // 2
    return make_lakes(size, size, seed, e_sigma=32.0, e_max=1500.0,
                      ignition_patch=(r0, r0, n), T=T)


def paper_plain(side, T=300, wind_speed=5.0, wind_dir=45.0):
    """The paper's timing workload shape (Sec. 3, forward prediction): a square
    plain landscape (flat, uniform neutral fuel) with fixed wind and a centre
    ignition, 300 steps."""
    z = np.zeros((side, side), dtype=np.float32)
    ign = np.zeros((side, side), dtype=np.uint8)
    ign[side // 2, side // 2] = 1
    s = Scenario(H=side, W=side, p_veg=z, p_den=z.copy(), elevation=z.copy(),
                 wind_speed=None, wind_dir=None,
                 wind_speed_scalar=float(np.float32(wind_speed)),
                 wind_dir_scalar=float(np.float32(wind_dir)),
                 init_burning=ign, seed=side, T=T)
    return s.with_params(*s.params)


def config3_sizes(n=256):
    """Grid sides (H_b, W_b) of the batched ensemble, log-uniform in [256, 2048]."""
    out = []
    for b in range(n):
        rng = np.random.default_rng(3000 + b)
        u = rng.random(2)
        out.append(tuple(int(round(256.0 * 8.0 ** x)) for x in u))
    return out


def config3_scenario(b, T=300, scale=1.0):
    """Scenario b of the batched ensemble: config-0 generators, +-20 % jitter.

    ``scale`` shrinks the sides (for tests); 1.0 is the benchmark workload.
    """
    rng = np.random.default_rng(3000 + b)
    u = rng.random(2)
    H, W = (max(8, int(round(256.0 * 8.0 ** x * scale))) for x in u)
    j = rng.uniform(0.8, 1.2, size=8)
    p = PARAMS_TRUE
    veg, den, elev = _base(rng, H, W, "iid", 0.05, 8.0, 300.0 * j[7])
    ign = _ignite(veg, [(H // 2, W // 2)])
    s = Scenario(H=H, W=W, p_veg=_f32(veg), p_den=_f32(den), elevation=_f32(elev),
                 wind_speed=None, wind_dir=None,
                 wind_speed_scalar=float(np.float32(5.0 * j[5])),
                 wind_dir_scalar=float(np.float32(45.0 * j[6])),
                 init_burning=ign, seed=3000 + b, scenario_id=b, T=T)
    return s.with_params(p[0] * j[0], p[1] * j[1], p[2] * j[2], p[3] * j[3],
                         P_CONTINUE * j[4])


def config4_scenario(b, size=1024, T=200):
    """Calibration scenario b: config-1 generators, target and start parameters.

    Returns (scenario with the true parameters, start parameters (p_h, a, c1, c2)).
    The target burn map is simulated with Philox seed 9000 + b.
    """
    s = make_lakes(size, size, 4000 + b, T=T, scenario_id=b)
    rng = np.random.default_rng(5000 + b)
    start = tuple(float(np.float32(v * f)) for v, f in
                  zip(PARAMS_TRUE, rng.uniform(0.6, 1.4, size=4)))
    s = dataclasses.replace(s, seed=9000 + b)
    return s, start


def synthetic_front_state(H, W, seed, *, n_fires=3, r_min=None, r_max=None,
                          front=2.0, noise=1.5, p_veg=None):
    """A plausible mid-run fire state: burned discs ringed by a burning front.

    Returns uint8 H x W with 0 = burnable, 1 = burning, 2 = burned.  Cells with
    p_veg = -1 (if given) are left burnable.  Used to start parity runs at full
    size without simulating from the ignition.
    """
    rng = np.random.default_rng(seed)
    r_min = r_min if r_min is not None else max(2.0, min(H, W) / 40)
    r_max = r_max if r_max is not None else max(r_min + 1, min(H, W) / 6)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    state = np.zeros((H, W), dtype=np.uint8)
    wobble = gaussian_filter(rng.standard_normal((H, W)), 4.0, mode="reflect")
    wobble = wobble / (np.abs(wobble).max() + 1e-12) * noise
    for _ in range(n_fires):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        rad = rng.uniform(r_min, r_max)
        d = np.hypot(yy - cy, xx - cx) + wobble
        state = np.where((d < rad - front) & (state == 0), 2, state)
        ring = (d >= rad - front) & (d < rad)
        state = np.where(ring & (state != 2), 1, state)
    sprinkle = rng.random((H, W)) < 0.02
    state = np.where(sprinkle & (state == 2), 1, state).astype(np.uint8)
    if p_veg is not None:
        state = np.where(p_veg <= -1.0, 0, state).astype(np.uint8)
    return np.ascontiguousarray(state)


def encode_planes(state):
    """uint8 {0,1,2} H x W -> 2 x H x W channels (burning, burned)."""
    out = np.zeros((2,) + state.shape, dtype=np.uint8)
    out[0] = state == 1
    out[1] = state == 2
    return out


def decode_planes(planes):
    """2 x H x W (burning, burned) -> uint8 {0,1,2}; raises on burning & burned."""
    b = planes[0].astype(bool)
    d = planes[1].astype(bool)
    if np.any(b & d):
        raise ValueError("cell both burning and burned")
    return (b.astype(np.uint8) + 2 * d.astype(np.uint8)).astype(np.uint8)
