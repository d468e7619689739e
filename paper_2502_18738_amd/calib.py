"""Calibration of (p_h, a, c1, c2) with the hand-written adjoint.

``FireCalib`` is a ``torch.autograd.Function``: its forward runs the CA in
calibration mode on the GPU and returns the accumulator y-hat (p_ignite at each
cell's ignition step, Sec. 2.2 data flow); its backward calls the library's
adjoint, which recomputes every checkpoint segment and returns
d(sum lambda * y-hat)/d theta with the sampled states held constant (Sec. 2.3).

``calibrate`` is the gradient-descent loop of Algorithm 1 for one observation
per epoch: a fresh seed per epoch (the epoch seed), forward, Eq. 10 loss and
its gradient (fused in the library), AdamW (lr 5e-3 by default, Sec. 2.3) and
the parameter clamps of Algorithm 1.
"""

from __future__ import annotations

from typing import Optional, Sequence

import torch

from ._abi import SIM_E_PARAM, SIM_LOSS_BCE, SimError
from .sim import Sim

# Clamp ranges of Algorithm 1: p_h in [0.2, 1], a, c1, c2 in [0, 1].
CLAMP_LO = (0.2, 0.0, 0.0, 0.0)
CLAMP_HI = (1.0, 1.0, 1.0, 1.0)


class FireCalib(torch.autograd.Function):
    """y-hat = FireCalib.apply(theta, sim, T, seeds).

    theta: (n, 4) tensor of (p_h, a, c1, c2) per scenario.  Returns the
    accumulators of all scenarios concatenated (flat FP32).  p_continue is
    taken from ``sim.p_continue`` and never differentiated.
    """

    @staticmethod
    def forward(ctx, theta: torch.Tensor, sim: Sim, T: int, seeds: Optional[Sequence[int]]):
        if not sim.calib:
            raise ValueError("FireCalib needs a Sim created with calib=True")
        p = theta.detach().to("cpu", torch.float32)
        rows = [tuple(r) + (pc,) for r, pc in zip(p.tolist(), sim.p_continue)]
        sim.set_params(rows)
        sim.reset(seeds)
        sim.run(int(T))
        ctx.sim = sim
        ctx.theta_dtype = theta.dtype
        return sim.accumulators()

    @staticmethod
    def backward(ctx, grad_yhat):
        g = ctx.sim.adjoint(grad_yhat.contiguous())
        return g.to(ctx.theta_dtype), None, None, None


def clamp_(theta: torch.Tensor) -> torch.Tensor:
    lo = torch.tensor(CLAMP_LO, dtype=theta.dtype, device=theta.device)
    hi = torch.tensor(CLAMP_HI, dtype=theta.dtype, device=theta.device)
    with torch.no_grad():
        theta.copy_(torch.maximum(torch.minimum(theta, hi), lo))
    return theta


def calibrate(sim: Sim, target, theta0, *, T: int, steps: int = 50, lr: float = 5e-3,
              loss_kind: int = SIM_LOSS_BCE, seed0: int = 1000, callback=None):
    """Gradient-descent calibration of every scenario of ``sim`` against
    ``target`` (uint8, the n grids concatenated).

    Returns (theta, history) where history holds (loss per scenario, theta)
    after every step.  Gradient step g uses Philox seed ``seed0 + g`` for all
    scenarios (a new epoch seed each step).  The parameters go to the library
    from device memory and the history stays on the device until the end, so
    the loop never waits for the host; a parameter row the library rejected
    (non-finite or p_h < 0) raises ``SimError`` after the loop.
    """
    theta = torch.as_tensor(theta0, dtype=torch.float32, device=sim.device).clone()
    theta.requires_grad_(True)
    opt = torch.optim.AdamW([theta], lr=lr)
    history = []
    y = torch.as_tensor(target, device=sim.device).to(torch.uint8).view(-1)
    for g in range(steps):
        sim.set_params_device(theta.detach())
        sim.reset([seed0 + g] * sim.n)
        sim.run(int(T))
        loss, grad = sim.loss_grad(y, loss_kind)
        theta.grad = grad.to(theta.dtype)
        opt.step()
        opt.zero_grad(set_to_none=True)
        clamp_(theta)
        history.append((loss.detach().clone(), theta.detach().clone()))
        if callback is not None:
            callback(g, loss, theta)
    bad = sim.params_rejected()
    if bad:
        raise SimError(SIM_E_PARAM, f"{bad} parameter rows were rejected during calibration "
                                    "(non-finite or p_h < 0)")
    return theta.detach(), [(l.cpu(), t.cpu()) for l, t in history]


def calibrate_sequence(sim: Sim, observations, theta0, *, interval: int, epochs: int = 1,
                       lr: float = 5e-3, loss_kind: int = SIM_LOSS_BCE, winds=None,
                       seed0: int = 1000):
    """Algorithm 1 with several observations per epoch.

    ``observations[it]`` (uint8, the n grids concatenated) is the observed
    fire after (it + 1) * interval steps; ``winds[it]`` (optional) is a list of
    (speed field or None, direction field or None, speed scalar, direction
    scalar) per scenario, set before the replay of iteration it.  Each epoch
    draws a new seed and keeps it for all of its iterations (Sec. 2.3); every
    iteration replays the fire from the start with the latest parameters,
    takes the Eq. 10 loss and its gradient, one AdamW step and the clamps.

    Returns (theta, history): one dict per iteration with ``epoch``,
    ``iteration``, ``loss`` (per scenario), ``grad`` (n x 4, the gradient the
    step used), ``theta`` (after the step and the clamps), ``jaccard`` (Eq. 11
    of the simulated and observed affected areas at the observation time,
    per scenario) and ``manhattan`` (Eq. 12: the sum over this epoch's
    observation times so far of the absolute difference of the affected-cell
    counts, per scenario).  The counts come from the device (sim.metrics).
    """
    theta = torch.as_tensor(theta0, dtype=torch.float32, device=sim.device).clone()
    theta.requires_grad_(True)
    opt = torch.optim.AdamW([theta], lr=lr)
    history = []
    for ep in range(epochs):
        seed = seed0 + ep
        manhattan = torch.zeros(sim.n, dtype=torch.int64)
        for it, obs in enumerate(observations):
            p = theta.detach().to("cpu")
            sim.set_params([tuple(r) + (pc,) for r, pc in zip(p.tolist(), sim.p_continue)])
            sim.reset([seed] * sim.n)
            if winds is not None:
                for s_, w in enumerate(winds[it]):
                    sim.set_wind(s_, *w)
            sim.run((it + 1) * int(interval))
            y = torch.as_tensor(obs, device=sim.device).to(torch.uint8).view(-1)
            m = sim.metrics(y).cpu()          # |A & B|, |A | B|, |A|, |B| per scenario
            loss, grad = sim.loss_grad(y, loss_kind)
            theta.grad = grad.to(theta.dtype)
            opt.step()
            opt.zero_grad(set_to_none=True)
            clamp_(theta)
            manhattan = manhattan + (m[:, 2] - m[:, 3]).abs()
            jac = torch.where(m[:, 1] > 0, m[:, 0].double() / m[:, 1].clamp(min=1).double(),
                              torch.ones(sim.n, dtype=torch.float64))
            history.append({"epoch": ep, "iteration": it, "loss": loss.detach().cpu(),
                            "grad": grad.detach().cpu(), "theta": theta.detach().cpu().clone(),
                            "jaccard": jac, "manhattan": manhattan.clone()})
    return theta.detach(), history
