"""Python handle over libfiresim (argument marshalling only).

PyTorch provides device memory and the stream; every step of the automaton
runs in the library's HIP kernels.
"""

from __future__ import annotations

import contextlib
import ctypes
from typing import Iterable, Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import SimError


def _dev_tensor(a, dtype, device):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)
    return t.contiguous()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Sim:
    """n wildfire scenarios advanced together on one GPU.

    ``scenarios``: objects with H, W, cell_m, seed, scenario_id, the fields
    p_veg, p_den, elevation, wind_speed, wind_dir (or None with the
    ``*_scalar`` values), init_burning and the parameters p_h, a, c1, c2,
    p_continue (numpy arrays or torch tensors).
    """

    def __init__(self, scenarios: Sequence, *, device="cuda", calib: bool = False,
                 stats: bool = False, ckpt_every: int = 20, T_max: Optional[int] = None,
                 tielog: bool = False,
                 exec: Optional[dict] = None, stream: Optional[torch.cuda.Stream] = None,
                 static_scratch: bool = False):
        self._lib = _abi.load()
        self.device = torch.device(device)
        self.n = len(scenarios)
        self.shapes = [(int(s.H), int(s.W)) for s in scenarios]
        self.offsets = np.concatenate([[0], np.cumsum([h * w for h, w in self.shapes])])
        self.calib = bool(calib)
        self.p_continue = [float(np.float32(s.p_continue)) for s in scenarios]
        flags = ((_abi.SIM_F_CALIB if calib else 0) | (_abi.SIM_F_STATS if stats else 0)
                 | (_abi.SIM_F_TIELOG if tielog else 0))
        if calib and T_max is None:
            T_max = max(int(getattr(s, "T", 0)) for s in scenarios)
        T_max = int(T_max or 0)
        self._keep = []
        self._h = None
        # static_scratch: the handle's workspace is the library's static array
        # on this device (sim_init_static), so construction allocates no
        # workspace; at most one such handle per device at a time
        self.static_scratch = bool(static_scratch)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with self._on_stream():
            self._init(scenarios, flags, int(ckpt_every), T_max)
        if exec is not None:
            self.set_exec(**exec)

    def _init(self, scenarios, flags, ckpt_every, T_max):
        descs = (_abi.sim_desc * self.n)()
        for i, s in enumerate(scenarios):
            f32 = lambda a: _dev_tensor(a, torch.float32, self.device)
            pv, pd, el = f32(s.p_veg), f32(s.p_den), f32(s.elevation)
            ws, wd = f32(s.wind_speed), f32(s.wind_dir)
            ign = _dev_tensor(s.init_burning, torch.uint8, self.device)
            sl = f32(getattr(s, "slope_deg", None))
            hw = int(s.H) * int(s.W)
            for name, t, k in (("p_veg", pv, 1), ("p_den", pd, 1), ("elevation", el, 1),
                               ("wind_speed", ws, 1), ("wind_dir", wd, 1),
                               ("init_burning", ign, 1), ("slope_deg", sl, 9)):
                if t is not None and t.numel() != k * hw:
                    raise ValueError(f"scenario {i}: {name} holds {t.numel()} values, "
                                     f"expected {k * hw}")
            self._keep += [pv, pd, el, ws, wd, ign, sl]
            fields = _abi.sim_fields(
                pv.data_ptr(), pd.data_ptr(), None if el is None else el.data_ptr(),
                None if ws is None else ws.data_ptr(), None if wd is None else wd.data_ptr(),
                float(s.wind_speed_scalar), float(s.wind_dir_scalar), ign.data_ptr(),
                None if sl is None else sl.data_ptr())
            par = _abi.sim_params(*(float(np.float32(getattr(s, k)))
                                    for k in ("p_h", "a", "c1", "c2", "p_continue")))
            descs[i] = _abi.sim_desc(int(s.H), int(s.W), float(s.cell_m),
                                     int(s.scenario_id) & 0xFFFFFFFF,
                                     int(s.seed) & 0xFFFFFFFFFFFFFFFF, par, fields)
        self._descs = descs
        h = ctypes.c_void_p()
        if self.static_scratch:
            self.workspace = None
            with torch.cuda.device(self.device):
                rc = self._lib.sim_init_static(ctypes.byref(h), descs, self.n,
                                               ctypes.c_void_p(self.stream.cuda_stream), flags,
                                               int(ckpt_every), T_max)
        else:
            nbytes = self._lib.sim_workspace_size(descs, self.n, flags, int(ckpt_every), T_max)
            if nbytes == 0:
                raise SimError(_abi.SIM_E_ARG, "invalid scenario descriptions")
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            rc = self._lib.sim_init(ctypes.byref(h), descs, self.n, ctypes.c_void_p(aligned),
                                    nbytes, ctypes.c_void_p(self.stream.cuda_stream), flags,
                                    int(ckpt_every), T_max)
        if rc != 0:
            raise SimError(rc, self._lib.sim_last_error(None).decode())
        self._h = h

    # ------------------------------------------------------------ plumbing
    def _check(self, rc):
        if rc != 0:
            raise SimError(rc, self._lib.sim_last_error(self._h).decode())

    @contextlib.contextmanager
    def _on_stream(self, inputs=(), outputs=()):
        """Run a library call on the handle's stream.  When the caller works on
        another stream: the handle's stream first waits for the caller's work
        (inputs it produced are complete), temporaries are allocated on the
        handle's stream, the caller's input tensors are marked as used there
        (the allocator does not hand their memory out while the library may
        still read them), and afterwards the caller's stream waits for the
        library's work and the outputs are marked as used on it."""
        cur = torch.cuda.current_stream(self.device)
        if cur == self.stream:
            yield
            return
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            yield
        for t in inputs:
            if isinstance(t, torch.Tensor) and t.is_cuda:
                t.record_stream(self.stream)
        cur.wait_stream(self.stream)
        for t in outputs:
            if isinstance(t, torch.Tensor) and t.is_cuda:
                t.record_stream(cur)

    def close(self):
        if getattr(self, "_h", None):
            # the workspace and fields are freed with this object: let the
            # handle's queued work finish first
            self.stream.synchronize()
            self._lib.sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- calls
    def set_exec(self, tile_rows=32, tile_words=2, depth=32, skip=1, threads=0):
        """skip: 0 process every tile, 1 (or True) device worklist, 2 per-tile test
        of the neighbours' flags, 3 every tile launched and tested against the
        worklist; threads: work-group size (0 = the shape's default)."""
        e = _abi.sim_exec(int(tile_rows), int(tile_words), int(depth), int(skip), int(threads))
        with self._on_stream():
            self._check(self._lib.sim_set_exec(self._h, ctypes.byref(e)))

    def get_exec(self):
        e = _abi.sim_exec()
        self._check(self._lib.sim_get_exec(self._h, ctypes.byref(e)))
        return dict(tile_rows=e.tile_rows, tile_words=e.tile_words, depth=e.depth,
                    skip=int(e.skip), threads=int(e.threads))

    def autotune(self, T_probe: int = 32) -> dict:
        """Time every compiled execution shape over T_probe steps from the
        current state (restored afterwards) and keep the fastest."""
        e = _abi.sim_exec()
        with self._on_stream():
            self._check(self._lib.sim_autotune(self._h, int(T_probe), ctypes.byref(e)))
        return dict(tile_rows=e.tile_rows, tile_words=e.tile_words, depth=e.depth,
                    skip=int(e.skip), threads=int(e.threads))

    def use_graphs(self, on: bool = True):
        self._check(self._lib.sim_use_graphs(self._h, int(bool(on))))

    def run(self, T: int):
        with self._on_stream():
            self._check(self._lib.sim_run(self._h, int(T)))

    def prepare(self, T: int):
        """Build the propagation table for the next T steps now (run() does it
        itself when needed)."""
        with self._on_stream():
            self._check(self._lib.sim_prepare(self._h, int(T)))

    def step(self):
        with self._on_stream():
            self._check(self._lib.sim_step(self._h))

    @property
    def t(self) -> int:
        v = ctypes.c_int32()
        self._check(self._lib.sim_get_step(self._h, ctypes.byref(v)))
        return v.value

    def set_params(self, params: Iterable):
        """params: n rows of (p_h, a, c1, c2, p_continue)."""
        rows = [tuple(float(x) for x in r) for r in params]
        arr = (_abi.sim_params * self.n)(*[_abi.sim_params(*r) for r in rows])
        with self._on_stream():
            self._check(self._lib.sim_set_params(self._h, arr))
        self.p_continue = [float(np.float32(r[4])) for r in rows]

    def set_params_device(self, theta: torch.Tensor):
        """theta: (n, 4) tensor of (p_h, a, c1, c2) on the handle's device,
        read by the library in stream order (no host round trip); p_continue
        is kept.  Rows the library rejects (non-finite, p_h < 0) keep their
        parameters and are counted by ``params_rejected``."""
        if not (isinstance(theta, torch.Tensor) and theta.is_cuda):
            raise ValueError("theta must be a CUDA tensor")
        if tuple(theta.shape) != (self.n, 4):
            raise ValueError("theta must have shape (n, 4)")
        with self._on_stream(inputs=[theta]):
            t = theta.detach().to(torch.float32).contiguous()
            self._check(self._lib.sim_set_params_device(self._h, _ptr(t)))

    def params_rejected(self) -> int:
        """Rows ``set_params_device`` rejected since the last call (waits for
        the handle's stream)."""
        out = ctypes.c_int32(0)
        self._check(self._lib.sim_params_rejected(self._h, ctypes.byref(out)))
        return int(out.value)

    def reset(self, seeds: Optional[Sequence[int]] = None):
        arr = None
        if seeds is not None:
            arr = (ctypes.c_uint64 * self.n)(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in seeds])
        with self._on_stream():
            self._check(self._lib.sim_reset(self._h, arr))

    def get_state(self, s: int = 0) -> torch.Tensor:
        H, W = self.shapes[s]
        out = torch.empty((2, H, W), dtype=torch.uint8, device=self.device)
        with self._on_stream(outputs=[out]):
            self._check(self._lib.sim_get_state(self._h, s, _ptr(out)))
        return out

    def set_state(self, s: int, planes, step: int):
        H, W = self.shapes[s]
        with self._on_stream(inputs=[planes]):
            t = _dev_tensor(planes, torch.uint8, self.device)
            if tuple(t.shape) != (2, H, W):
                raise ValueError(f"state must be 2 x {H} x {W}")
            self._check(self._lib.sim_set_state(self._h, s, _ptr(t), int(step)))
            self.stream.synchronize()

    def pignite(self, s: int = 0) -> torch.Tensor:
        H, W = self.shapes[s]
        out = torch.empty((H, W), dtype=torch.float32, device=self.device)
        with self._on_stream(outputs=[out]):
            self._check(self._lib.sim_pignite(self._h, s, _ptr(out)))
        return out

    def accumulator(self, s: int = 0) -> torch.Tensor:
        H, W = self.shapes[s]
        out = torch.empty((H, W), dtype=torch.float32, device=self.device)
        with self._on_stream(outputs=[out]):
            self._check(self._lib.sim_accumulator(self._h, s, _ptr(out)))
        return out

    def accumulators(self) -> torch.Tensor:
        """All accumulators concatenated (flat FP32, the adjoint's layout)."""
        out = torch.empty(int(self.offsets[-1]), dtype=torch.float32, device=self.device)
        with self._on_stream(outputs=[out]):
            for s in range(self.n):
                a, b = int(self.offsets[s]), int(self.offsets[s + 1])
                self._check(self._lib.sim_accumulator(self._h, s, _ptr(out[a:b])))
        return out

    def set_adjoint(self, method: str = "checkpoint", rings=None):
        """method: "checkpoint" (recompute segments) or "timemap"; rings:
        None (every step attached) or (r_first, r_between, r_last)."""
        m = {"checkpoint": _abi.SIM_ADJ_CHECKPOINT, "timemap": _abi.SIM_ADJ_TIMEMAP}[method]
        rf, rb, rl = (-1, 0, 0) if rings is None else (int(x) for x in rings)
        self._check(self._lib.sim_set_adjoint(self._h, m, rf, rb, rl))

    def adjoint(self, dL_dyhat: torch.Tensor) -> torch.Tensor:
        grad = torch.empty((self.n, 4), dtype=torch.float64, device=self.device)
        with self._on_stream(inputs=[dL_dyhat], outputs=[grad]):
            lam = dL_dyhat.to(device=self.device, dtype=torch.float32).contiguous().view(-1)
            if lam.numel() != int(self.offsets[-1]):
                raise ValueError("dL_dyhat must hold every scenario's grid, concatenated")
            self._check(self._lib.sim_adjoint(self._h, _ptr(lam), _ptr(grad)))
        return grad

    def loss_grad(self, target, kind: int = _abi.SIM_LOSS_BCE):
        loss = torch.empty(self.n, dtype=torch.float64, device=self.device)
        grad = torch.empty((self.n, 4), dtype=torch.float64, device=self.device)
        with self._on_stream(inputs=[target], outputs=[loss, grad]):
            y = _dev_tensor(target, torch.uint8, self.device).view(-1)
            if y.numel() != int(self.offsets[-1]):
                raise ValueError("target must hold every scenario's grid, concatenated")
            self._check(self._lib.sim_loss_grad(self._h, _ptr(y), int(kind), _ptr(loss),
                                                _ptr(grad)))
        return loss, grad

    def set_wind(self, s: int, wind_speed=None, wind_dir=None, speed_scalar=0.0, dir_scalar=0.0):
        """New wind for scenario s (fields H x W, or None for the scalars)."""
        with self._on_stream(inputs=[wind_speed, wind_dir]):
            ws = _dev_tensor(wind_speed, torch.float32, self.device)
            wd = _dev_tensor(wind_dir, torch.float32, self.device)
            hw = self.shapes[s][0] * self.shapes[s][1] if 0 <= s < self.n else 0
            for t in (ws, wd):
                if t is not None and t.numel() != hw:
                    raise ValueError("wind fields must hold H*W values of scenario s")
            self._check(self._lib.sim_set_wind(self._h, int(s), _ptr(ws), _ptr(wd),
                                               float(speed_scalar), float(dir_scalar)))

    def ignite(self, s: int, cells):
        """Spotting: set cells (flat r*W + c indices) burning before the next step."""
        with self._on_stream(inputs=[cells]):
            c = _dev_tensor(np.asarray(cells, dtype=np.int32)
                            if not isinstance(cells, torch.Tensor) else cells,
                            torch.int32, self.device).view(-1)
            self._check(self._lib.sim_ignite(self._h, int(s), _ptr(c), int(c.numel())))

    def counts(self) -> torch.Tensor:
        """(n, 2) int64 device tensor: burning and burned cells per scenario."""
        out = torch.empty((self.n, 2), dtype=torch.int64, device=self.device)
        with self._on_stream(outputs=[out]):
            self._check(self._lib.sim_counts(self._h, _ptr(out)))
        return out

    def overlap(self, s: int, target) -> torch.Tensor:
        """(|A & B|, |A | B|) of scenario s's affected cells and a target mask."""
        out = torch.empty(2, dtype=torch.int64, device=self.device)
        with self._on_stream(inputs=[target], outputs=[out]):
            y = _dev_tensor(target, torch.uint8, self.device)
            if not 0 <= s < self.n or y.numel() != self.shapes[s][0] * self.shapes[s][1]:
                raise ValueError("target must hold H*W values of scenario s")
            self._check(self._lib.sim_overlap(self._h, int(s), _ptr(y), _ptr(out)))
        return out

    def jaccard(self, s: int, target) -> float:
        """Eq. 11 against a target affected-area mask."""
        i, u = (int(x) for x in self.overlap(s, target).cpu())
        return 1.0 if u == 0 else i / u

    def metrics(self, targets) -> torch.Tensor:
        """(n, 4) int64 device tensor: per scenario (|A & B|, |A | B|, |A|, |B|)
        of its affected cells A and its observed map B (``targets``: the n
        grids concatenated) -- the inputs of Eq. 11 and Eq. 12."""
        out = torch.empty((self.n, 4), dtype=torch.int64, device=self.device)
        with self._on_stream(inputs=[targets], outputs=[out]):
            y = _dev_tensor(targets, torch.uint8, self.device).view(-1)
            if y.numel() != int(self.offsets[-1]):
                raise ValueError("targets must hold every scenario's grid, concatenated")
            self._check(self._lib.sim_metrics(self._h, _ptr(y), _ptr(out)))
        return out

    def arrival(self, s0: int = 0, n: Optional[int] = None, counts=None) -> torch.Tensor:
        """Add, per cell, the number of scenarios s0 .. s0+n-1 (one grid shape)
        in which the cell is affected to ``counts`` (uint32-compatible int32
        H x W device tensor, created zeroed when None) and return it."""
        n = self.n - s0 if n is None else int(n)
        if not 0 <= s0 < self.n:
            raise ValueError("s0 out of range")
        H, W = self.shapes[s0]
        if counts is None:
            counts = torch.zeros((H, W), dtype=torch.int32, device=self.device)
        if counts.dtype != torch.int32 or counts.numel() != H * W or not counts.is_contiguous():
            raise ValueError("counts must be a contiguous int32 tensor of H*W cells")
        with self._on_stream(inputs=[counts], outputs=[counts]):
            self._check(self._lib.sim_arrival(self._h, int(s0), n, _ptr(counts)))
        return counts

    def tie_log(self):
        """Near-tie records logged since the last reset (handle created with
        tielog=True): a numpy structured array with fields scenario, step,
        cell, p_ignite, draw, ignited, sorted by (scenario, step, cell); and the
        number of trials logged (more than the records if the log overflowed)."""
        n = ctypes.c_int64()
        with self._on_stream():
            self._check(self._lib.sim_tielog(self._h, None, 0, ctypes.byref(n)))
            m = min(int(n.value), _abi.SIM_TIELOG_CAP)
            buf = torch.empty(max(m, 1) * ctypes.sizeof(_abi.sim_tie), dtype=torch.uint8,
                              device=self.device)
            self._check(self._lib.sim_tielog(self._h, _ptr(buf), m, ctypes.byref(n)))
        dt = np.dtype([("scenario", "<i4"), ("step", "<i4"), ("cell", "<i8"),
                       ("p_ignite", "<f4"), ("draw", "<f4"), ("ignited", "<i4"),
                       ("reserved", "<i4")])
        rec = buf[: m * dt.itemsize].cpu().numpy().view(dt)
        rec = np.sort(rec, order=["scenario", "step", "cell"])
        return rec, int(n.value)

    def stats(self) -> dict:
        v = (ctypes.c_uint64 * 4)()
        self._check(self._lib.sim_stats(self._h, v))
        return dict(tiles=int(v[0]), trials=int(v[1]), ties=int(v[2]), launches=int(v[3]))


def ensemble_arrival(scenario, seeds: Sequence[int], T: int, *, batch: Optional[int] = None,
                     exec: Optional[dict] = None) -> torch.Tensor:
    """Probability of arrival (Sec. 1): the fraction of runs, one per seed, in
    which each cell is affected after T steps.  Runs go in batches of
    ``batch`` scenarios (all of them at once by default) through one handle
    per batch; returns an FP32 H x W device tensor."""
    import dataclasses

    seeds = [int(x) for x in seeds]
    if not seeds:
        raise ValueError("need at least one seed")
    batch = len(seeds) if batch is None else max(1, int(batch))
    counts = None
    for b0 in range(0, len(seeds), batch):
        part = [dataclasses.replace(scenario, seed=sd) for sd in seeds[b0:b0 + batch]]
        sim = Sim(part, exec=exec)
        sim.run(int(T))
        counts = sim.arrival(0, len(part), counts)
        del sim
    return counts.to(torch.float32) / float(len(seeds))
