"""FP64 CPU oracle for the chi(2) split-step Fourier z-loop of BRAHMS.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP engine.

It is a plain, slow, literal statement of the method of the paper
(arXiv 2609.08384), written in complex128 with PyTorch CPU tensors (the FFT and
elementwise products are library primitives; there is no blocking, fusion or
reordering beyond what the method states):

* coupled equations (Sec. 2, eqs. CEp/CEs/CEi) in the matrix form of
  Sec. 3.1 (eq. CWEsmatrix): dA/dz = (L + N) A with L diagonal (dispersion,
  diffraction, walk-off, absorption) and N the chi(2) coupling with the
  exp(-/+ i dk z) mismatch phase;
* symmetric splitting N/2 - L - N/2 (Sec. 3.1, eq. expon), the linear step
  done in Fourier space by a forward and an inverse transform, the nonlinear
  half-steps by a classical fourth-order Runge-Kutta step (Sec. 3.1);
* as a second reference, the same splitting repeated over several steps with
  each pair of adjacent nonlinear half-steps taken as one Runge-Kutta step of
  size dz (Oracle.propagate_merged): eq. expon repeated puts two half-step
  flows of N next to each other, and the exact flows of one ODE over
  adjacent intervals compose to the flow over their union, so only the
  Runge-Kutta truncation term differs from the literal splitting.

Readings of passages that are silent or inconsistent (each is listed in the
design notes of the repository):

* diffraction enters as +i D (d2/dx2 + d2/dy2) with D = 1/(2k): this is the
  sign for which the focused entrance beam of eq. gaussianbeamc focuses at
  the crystal centre and for which the Boyd-Kleinman optimum falls at a
  negative dk (Sec. 5.2); eq. diffOp prints the opposite sign;
* walk-off is -tan(rho) d/dx, group delay -delta d/dtau (delta given
  directly), GVD -i (k''/2) d2/dtau2 (eq. dispOp), third-order dispersion
  +(k'''/6) d3/dtau3 (the Taylor coefficient; eq. dispOp prints a
  non-unitary i k'''/3), absorption -alpha/2;
* the mismatch phase is Phi(z) = integral of dk from 0 to z with dk piecewise
  constant per z-step (reduces to dk*z for a constant dk);
* SHG is the degenerate two-field system (index 0 = fundamental F,
  index 1 = second harmonic S):
      dF/dz = L_F F + i kappa_F S F* exp(+i Phi),
      dS/dz = L_S S + i kappa_S F^2  exp(-i Phi);
* periodic boundaries in x, y and tau; grid coordinates
  x_a = (a - floor(n/2)) dx; forward transform exp(-2 pi i j k / n),
  angular frequencies 2 pi fftfreq(n, d) (the Nyquist bin negative).

Field arrays are complex tensors of shape [nt, ny, nx] (x fastest), one per
field, matching the x -> y -> tau index hierarchy of Sec. 4.3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import torch

DTYPE_R = torch.float64
DTYPE_C = torch.complex128


@dataclass
class FieldParams:
    """Linear and coupling coefficients of one field (eqs. dispOp, diffOp, CEx).

    Units are normalised: x, y, tau in grid cells, z in crystal lengths.
    """
    kappa: float = 0.0        # nonlinear coupling kappa_j
    diffraction: float = 0.0  # D_j = 1/(2 k_j)
    tan_rho: float = 0.0      # spatial walk-off tan(rho_j)
    delay: float = 0.0        # group-delay coefficient delta_j
    k2: float = 0.0           # GVD k''_j
    k3: float = 0.0           # TOD k'''_j
    alpha: float = 0.0        # linear (power) attenuation alpha_j


@dataclass
class Problem:
    """One propagation problem on an nx x ny x nt grid with nf = 2 or 3 fields."""
    nx: int
    ny: int
    nt: int
    nf: int
    dz: float
    fields: List[FieldParams]
    dk_const: float = 0.0
    dk: Optional[Sequence[float]] = None   # per-step dk_n (piecewise constant)
    dx: float = 1.0
    dy: float = 1.0
    dt: float = 1.0
    # transverse mismatch map: dk(x, y, z) = dk_n + s_n dk_map[y, x] in step n
    dk_map: Optional[object] = None        # [ny, nx] array (1/L), or None
    dk_map_scale: Optional[Sequence[float]] = None   # s_n per step (None: all 1)


# ---------------------------------------------------------------------------
# grid (periodic; coordinates centred on floor(n/2))
# ---------------------------------------------------------------------------

def axis_coords(n: int, d: float = 1.0) -> torch.Tensor:
    return (torch.arange(n, dtype=DTYPE_R) - (n // 2)) * d


def angular_freqs(n: int, d: float = 1.0) -> torch.Tensor:
    """2 pi fftfreq(n, d): the angular frequency of each transform bin."""
    m = torch.arange(n, dtype=DTYPE_R)
    m = torch.where(m >= (n + 1) // 2, m - n, m)  # Nyquist bin -> negative
    return 2.0 * math.pi * m / (n * d)


# ---------------------------------------------------------------------------
# linear operator L_j (eqs. dispOp + diffOp) and its Fourier symbol
# ---------------------------------------------------------------------------

def linear_symbol(fp: FieldParams, prob: Problem) -> torch.Tensor:
    """Symbol Lambda_j(kx, ky, w) of L_j, shape [nt, ny, nx].

    Derivatives map to multipliers d/dx -> i kx, d/dy -> i ky, d/dtau -> i w,
    so that L_j = i D (dxx + dyy) - tan(rho) dx - delta dtau
                  - i (k''/2) dtautau + (k'''/6) dtautautau - alpha/2
    becomes a multiplication in the transform domain.
    """
    kx = angular_freqs(prob.nx, prob.dx).view(1, 1, -1)
    ky = angular_freqs(prob.ny, prob.dy).view(1, -1, 1)
    w = angular_freqs(prob.nt, prob.dt).view(-1, 1, 1)
    ikx, iky, iw = 1j * kx, 1j * ky, 1j * w
    lam = (1j * fp.diffraction * (ikx ** 2 + iky ** 2)
           - fp.tan_rho * ikx
           - fp.delay * iw
           - 1j * (fp.k2 / 2.0) * iw ** 2
           + (fp.k3 / 6.0) * iw ** 3
           - fp.alpha / 2.0)
    return lam.to(DTYPE_C)


def fft3(a: torch.Tensor) -> torch.Tensor:
    return torch.fft.fftn(a, dim=(-3, -2, -1))


def ifft3(a: torch.Tensor) -> torch.Tensor:
    return torch.fft.ifftn(a, dim=(-3, -2, -1))


def linear_step(a: torch.Tensor, lam: torch.Tensor, dz: float) -> torch.Tensor:
    """exp(L dz) A = F^-1{ exp(Lambda dz) F{A} }  (Sec. 3.1)."""
    return ifft3(torch.exp(lam * dz) * fft3(a))


def linear_step_two_stage(a: torch.Tensor, fp: FieldParams, prob: Problem,
                          dz: float) -> torch.Tensor:
    """The paper's own linear sub-steps (Sec. 4.3): dispersion by 1D
    transforms along tau, then diffraction and walk-off by 2D transforms per
    tau-slice.  Equal to linear_step because the two operators commute."""
    w = angular_freqs(prob.nt, prob.dt).view(-1, 1, 1)
    iw = 1j * w
    lam_t = (-fp.delay * iw - 1j * (fp.k2 / 2.0) * iw ** 2
             + (fp.k3 / 6.0) * iw ** 3 - fp.alpha / 2.0)
    a = torch.fft.ifft(torch.exp(lam_t * dz) * torch.fft.fft(a, dim=0), dim=0)
    kx = angular_freqs(prob.nx, prob.dx).view(1, 1, -1)
    ky = angular_freqs(prob.ny, prob.dy).view(1, -1, 1)
    ikx, iky = 1j * kx, 1j * ky
    lam_xy = 1j * fp.diffraction * (ikx ** 2 + iky ** 2) - fp.tan_rho * ikx
    return torch.fft.ifft2(torch.exp(lam_xy * dz) * torch.fft.fft2(a, dim=(1, 2)),
                           dim=(1, 2))


# ---------------------------------------------------------------------------
# mismatch phase Phi(z) = int_0^z dk(z') dz'
# ---------------------------------------------------------------------------

def _piecewise_integral(values: Sequence[float], dz: float) -> Callable[[float], float]:
    """z -> integral_0^z v(z') dz' for v piecewise constant per step (v_n on
    [n dz, (n+1) dz))."""
    vals = [float(v) for v in values]
    cum = [0.0]
    for v in vals:
        cum.append(cum[-1] + v * dz)

    def integral(z: float) -> float:
        n = int(math.floor(z / dz + 1e-9))
        n = min(max(n, 0), len(vals) - 1)
        return cum[n] + vals[n] * (z - n * dz)
    return integral


def phase_function(prob: Problem) -> Callable:
    """Phi(z) = int_0^z dk dz' (reading of Sec. 2's exp(-/+ i dk z) for a dk
    that varies along z).  With a transverse map, dk(x, y, z) = dk_n +
    s_n dk_map(x, y) and Phi(x, y, z) = Phi(z) + dk_map(x, y) Psi(z),
    Psi(z) = int_0^z s dz' (a real [1, ny, nx] tensor for each z)."""
    if prob.dk is None:
        dk = float(prob.dk_const)
        base = lambda z: dk * z
    else:
        base = _piecewise_integral(prob.dk, prob.dz)
    if prob.dk_map is None:
        return base
    m = torch.as_tensor(prob.dk_map, dtype=DTYPE_R).reshape(1, prob.ny, prob.nx)
    if prob.dk_map_scale is None:
        psi = lambda z: z
    else:
        psi = _piecewise_integral(prob.dk_map_scale, prob.dz)
    return lambda z: base(z) + m * psi(z)


# ---------------------------------------------------------------------------
# nonlinear operator N (eqs. CEp/CEs/CEi) and the RK4 half-step
# ---------------------------------------------------------------------------

def _unit(phi):
    """exp(i phi) for a float or a (differentiable) real tensor phi."""
    if isinstance(phi, torch.Tensor):
        return torch.polar(torch.ones_like(phi), phi)
    return complex(math.cos(phi), math.sin(phi))


def nonlinear_rhs(a: List[torch.Tensor], phi,
                  prob: Problem) -> List[torch.Tensor]:
    """Right-hand side of the nonlinear part alone, at mismatch phase phi
    (a float, or a real tensor when gradients in phi are wanted)."""
    e_m = _unit(-phi)   # exp(-i Phi)
    e_p = _unit(phi)    # exp(+i Phi)
    k = [fp.kappa for fp in prob.fields]
    if prob.nf == 3:
        ap, as_, ai = a
        return [1j * k[0] * as_ * ai * e_m,
                1j * k[1] * ap * torch.conj(ai) * e_p,
                1j * k[2] * ap * torch.conj(as_) * e_p]
    f, s = a
    return [1j * k[0] * s * torch.conj(f) * e_p,
            1j * k[1] * f * f * e_m]


def rk4(a: List[torch.Tensor], z: float, h: float, prob: Problem,
        phi: Callable) -> List[torch.Tensor]:
    """One classical RK4 step of size h for dA/dz = N(A, z), starting at z."""
    def f(y, zz):
        return nonlinear_rhs(y, phi(zz), prob)

    k1 = f(a, z)
    k2 = f([y + (h / 2) * k for y, k in zip(a, k1)], z + h / 2)
    k3 = f([y + (h / 2) * k for y, k in zip(a, k2)], z + h / 2)
    k4 = f([y + h * k for y, k in zip(a, k3)], z + h)
    return [y + (h / 6) * (q1 + 2 * q2 + 2 * q3 + q4)
            for y, q1, q2, q3, q4 in zip(a, k1, k2, k3, k4)]


# ---------------------------------------------------------------------------
# the z-loop: N/2 - L - N/2 (eq. expon)
# ---------------------------------------------------------------------------

class Oracle:
    def __init__(self, prob: Problem):
        if prob.nf not in (2, 3) or len(prob.fields) != prob.nf:
            raise ValueError("nf must be 2 or 3 with one FieldParams per field")
        self.prob = prob
        self.lam = [linear_symbol(fp, prob) for fp in prob.fields]
        self.phi = phase_function(prob)

    def step(self, a: List[torch.Tensor], n: int) -> List[torch.Tensor]:
        """Step n: from z_n = n dz to z_{n+1}."""
        p = self.prob
        h = p.dz / 2
        z = n * p.dz
        a = rk4(a, z, h, p, self.phi)
        a = [linear_step(aj, lj, p.dz) for aj, lj in zip(a, self.lam)]
        a = rk4(a, z + h, h, p, self.phi)
        return a

    def propagate(self, a: List[torch.Tensor], nsteps: int,
                  n0: int = 0) -> List[torch.Tensor]:
        a = [torch.as_tensor(x).to(DTYPE_C).clone() for x in a]
        for n in range(n0, n0 + nsteps):
            a = self.step(a, n)
        return a

    def propagate_merged(self, a: List[torch.Tensor], nsteps: int,
                         n0: int = 0) -> List[torch.Tensor]:
        """Steps n0 .. n0 + nsteps - 1 of eq. expon with adjacent nonlinear
        half-steps merged: the first half-step of step n0, then per step the
        linear step over dz followed by one RK4 step of size dz from
        z_n + dz/2 (it covers the second half of step n and the first half of
        step n + 1), except after the last step, which ends with its own
        second half-step of size dz/2."""
        p = self.prob
        h = p.dz / 2
        a = [torch.as_tensor(x).to(DTYPE_C).clone() for x in a]
        if nsteps <= 0:
            return a
        a = rk4(a, n0 * p.dz, h, p, self.phi)
        for n in range(n0, n0 + nsteps):
            a = [linear_step(aj, lj, p.dz) for aj, lj in zip(a, self.lam)]
            size = h if n == n0 + nsteps - 1 else p.dz
            a = rk4(a, n * p.dz + h, size, p, self.phi)
        return a


def propagate(fields, prob: Problem, nsteps: int, n0: int = 0):
    return Oracle(prob).propagate(fields, nsteps, n0)


def propagate_merged(fields, prob: Problem, nsteps: int, n0: int = 0):
    return Oracle(prob).propagate_merged(fields, nsteps, n0)


# ---------------------------------------------------------------------------
# diagnostics: energies (Sec. 6 power integral summed over tau) and the
# Manley-Rowe combinations that the lossless equations conserve
# ---------------------------------------------------------------------------

def power_traces(a: List[torch.Tensor], prob: Problem) -> List[torch.Tensor]:
    """P_j(tau) = sum over x, y of |A_j|^2 dx dy: the pulse power per time
    slice, the output quantity plotted in Sec. 6 (fields are [nt, ny, nx])."""
    return [(x.abs() ** 2).sum(dim=(1, 2)) * (prob.dx * prob.dy) for x in a]


def energies(a: List[torch.Tensor], prob: Problem) -> List[float]:
    cell = prob.dx * prob.dy * prob.dt
    return [float((x.abs() ** 2).sum()) * cell for x in a]


def manley_rowe(a: List[torch.Tensor], prob: Problem) -> List[float]:
    e = energies(a, prob)
    k = [fp.kappa for fp in prob.fields]
    if prob.nf == 3:
        return [e[0] / k[0] + e[1] / k[1],
                e[0] / k[0] + e[2] / k[2],
                e[1] / k[1] - e[2] / k[2]]
    return [e[0] / k[0] + e[1] / k[1]]
