"""Gradients of the FP64 oracle's z-loop (test infrastructure only).

The oracle's own adjoint: reverse-mode automatic differentiation (PyTorch
autograd, complex128) through the literal forward loop of oracle/ssfm.py,
with the mismatch phase Phi(z) = int_0^z dk written as a differentiable
function of the per-step profile dk_n.  Each z-step is recomputed during the
backward sweep from its stored input (one checkpoint per step), so memory is
one state per step.  Complex gradients follow PyTorch's convention
dJ/dRe + i dJ/dIm for a real loss J.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import torch
from torch.utils.checkpoint import checkpoint

from . import ssfm


def _phase_tensor(dk: torch.Tensor, dz: float):
    """Phi(z) for a piecewise-constant profile dk (one entry per step)."""
    cum = torch.cat([dk.new_zeros(1), torch.cumsum(dk * dz, 0)])

    def phi(n: int, offset: float):
        return cum[n] + dk[n] * offset
    return phi


def _step(fields: List[torch.Tensor], dk: torch.Tensor, n: int, prob: ssfm.Problem,
          lam: List[torch.Tensor]) -> List[torch.Tensor]:
    """Step n of the N/2 - L - N/2 loop with a tensor-valued phase."""
    phi_n = _phase_tensor(dk, prob.dz)
    h = prob.dz / 2
    zn = n * prob.dz
    # rk4 evaluates the phase at absolute z; map z to (step, offset) of step n
    phase = lambda z: phi_n(n, z - zn)
    a = ssfm.rk4(fields, zn, h, prob, phase)
    a = [ssfm.linear_step(x, l, prob.dz) for x, l in zip(a, lam)]
    return ssfm.rk4(a, zn + h, h, prob, phase)


def forward(fields_in: Sequence[torch.Tensor], dk: torch.Tensor, prob: ssfm.Problem,
            nsteps: int) -> List[torch.Tensor]:
    """Differentiable forward loop from z = 0 (dk has >= nsteps entries)."""
    lam = [ssfm.linear_symbol(fp, prob) for fp in prob.fields]
    a = list(fields_in)
    for n in range(nsteps):
        packed = checkpoint(lambda *t, n=n: tuple(_step(list(t[:-1]), t[-1], n, prob, lam)),
                            *a, dk, use_reentrant=False)
        a = list(packed)
    return a


def shg_energy_loss(out: List[torch.Tensor], prob: ssfm.Problem) -> torch.Tensor:
    """J = - sum |S(x, y, tau, L)|^2 (cell volume included): minimising J
    maximises the generated second-harmonic energy (Sec. 6 power integral)."""
    cell = prob.dx * prob.dy * prob.dt
    return -(out[1].abs() ** 2).sum() * cell


def gradients(fields_in: Sequence, dk: Sequence[float], prob: ssfm.Problem, nsteps: int,
              loss=shg_energy_loss) -> Tuple[float, List[torch.Tensor], torch.Tensor]:
    """(J, dJ/dA_in per field, dJ/ddk_n) by reverse-mode differentiation."""
    if prob.dk_map is not None:
        raise NotImplementedError("gradients with a transverse mismatch map")
    a = [torch.as_tensor(x).to(ssfm.DTYPE_C).clone().requires_grad_(True) for x in fields_in]
    d = torch.as_tensor(list(dk), dtype=ssfm.DTYPE_R).clone().requires_grad_(True)
    out = forward(a, d, prob, nsteps)
    j = loss(out, prob)
    grads = torch.autograd.grad(j, a + [d])
    return float(j.detach()), [g.detach() for g in grads[:-1]], grads[-1].detach()


def loss_value(fields_in: Sequence, dk: Sequence[float], prob: ssfm.Problem, nsteps: int,
               loss=shg_energy_loss) -> float:
    with torch.no_grad():
        a = [torch.as_tensor(x).to(ssfm.DTYPE_C) for x in fields_in]
        d = torch.as_tensor(list(dk), dtype=ssfm.DTYPE_R)
        lam = [ssfm.linear_symbol(fp, prob) for fp in prob.fields]
        for n in range(nsteps):
            a = _step(a, d, n, prob, lam)
        return float(loss(a, prob))
