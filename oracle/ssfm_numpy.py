"""A second, independent FP64 oracle of the chi(2) split-step z-loop, in NumPy.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module; it shares no code with the HIP engine, nor with the
PyTorch oracle (oracle/ssfm.py), which it exists to cross-check: the two are
written separately from the paper (arXiv 2609.08384) and must agree to
rounding on small random problems.

What it computes (the same readings as oracle/ssfm.py, stated here again):

* state: nf = 2 (SHG: F, S) or 3 (p, s, i) complex128 arrays [nt, ny, nx];
* one z-step n (Sec. 3.1, eq. expon): a fourth-order Runge-Kutta step of
  size dz/2 for the nonlinear part alone (eqs. CEp/CEs/CEi, or the
  degenerate SHG pair), the linear part exactly in the transform domain over
  dz, and a second Runge-Kutta step of size dz/2;
* linear part (eqs. dispOp, diffOp with the readings of the repository: +i D
  transverse Laplacian, -tan(rho) d/dx, -delta d/dtau, -i k''/2 d2/dtau2,
  +k'''/6 d3/dtau3, -alpha/2), periodic in x, y, tau: the transform-domain
  factor is separable, exp(dz (X(kx) + Y(ky) + T(w))), built here as an
  outer product of one-axis factors, with kx = 2 pi fftfreq(nx, dx) etc.;
* mismatch phase: within step n the phase at z is Phi_n + dk_n (z - z_n)
  with Phi_n the sum of dk_m dz over earlier steps (dk constant per step);
  a transverse map adds m(x, y) (Psi_n + s_n (z - z_n)) the same way.
"""
from __future__ import annotations

import numpy as np


def _freqs(n: int, d: float) -> np.ndarray:
    return 2.0 * np.pi * np.fft.fftfreq(n, d)


class NumpyOracle:
    """Literal N/2 - L - N/2 loop for one problem.

    params: list of nf dicts with keys kappa, diffraction, tan_rho, delay,
    k2, k3, alpha (missing keys are 0).  dk: per-step profile or None (then
    dk_const).  dk_map: [ny, nx] or None, dk_map_scale: per-step s_n or None
    (then 1)."""

    def __init__(self, nx, ny, nt, params, dz, dk_const=0.0, dk=None, dx=1.0, dy=1.0, dt=1.0,
                 dk_map=None, dk_map_scale=None):
        self.shape = (nt, ny, nx)
        self.nf = len(params)
        if self.nf not in (2, 3):
            raise ValueError("two or three fields")
        self.dz = float(dz)
        self.kappa = [float(p.get("kappa", 0.0)) for p in params]
        kx, ky, w = _freqs(nx, dx), _freqs(ny, dy), _freqs(nt, dt)
        self.prop = []
        for p in params:
            g = lambda k: float(p.get(k, 0.0))  # noqa: E731
            # one-axis exponents of L (i d/dx -> -kx ... written out as i times the
            # multiplier of each derivative: d/dx -> i kx)
            ex = 1j * g("diffraction") * (-(kx ** 2)) - g("tan_rho") * (1j * kx)
            ey = 1j * g("diffraction") * (-(ky ** 2))
            et = (-g("delay") * (1j * w) - 1j * (g("k2") / 2.0) * (-(w ** 2))
                  + (g("k3") / 6.0) * (-1j * w ** 3) - g("alpha") / 2.0)
            fx, fy, ft = np.exp(self.dz * ex), np.exp(self.dz * ey), np.exp(self.dz * et)
            self.prop.append(ft[:, None, None] * fy[None, :, None] * fx[None, None, :])
        self.dk_const = float(dk_const)
        self.dk = None if dk is None else np.asarray(dk, dtype=np.float64)
        self.map = None if dk_map is None else np.asarray(dk_map, dtype=np.float64)[None, :, :]
        self.scale = None if dk_map_scale is None else np.asarray(dk_map_scale, dtype=np.float64)

    # -- mismatch phase inside step n at offset o in [0, dz] from z_n --------
    def _phase(self, n: int, o: float):
        if self.dk is None:
            ph = self.dk_const * (n * self.dz + o)
        else:
            ph = float(np.sum(self.dk[:n]) * self.dz) + self.dk[n] * o
        if self.map is None:
            return ph
        if self.scale is None:
            psi = n * self.dz + o
        else:
            psi = float(np.sum(self.scale[:n]) * self.dz) + self.scale[n] * o
        return ph + self.map * psi

    def _rhs(self, a, ph):
        em, ep = np.exp(-1j * ph), np.exp(1j * ph)
        k = self.kappa
        if self.nf == 3:
            p, s, i = a
            return [1j * k[0] * s * i * em, 1j * k[1] * p * np.conj(i) * ep, 1j * k[2] * p * np.conj(s) * ep]
        f, s = a
        return [1j * k[0] * s * np.conj(f) * ep, 1j * k[1] * f * f * em]

    def _rk4(self, a, n, o0, h):
        """One classical RK4 step of size h from z_n + o0 (stages at o0,
        o0 + h/2, o0 + h)."""
        def add(y, c, d):
            return [yy + c * dd for yy, dd in zip(y, d)]
        d1 = self._rhs(a, self._phase(n, o0))
        d2 = self._rhs(add(a, h / 2, d1), self._phase(n, o0 + h / 2))
        d3 = self._rhs(add(a, h / 2, d2), self._phase(n, o0 + h / 2))
        d4 = self._rhs(add(a, h, d3), self._phase(n, o0 + h))
        return [y + (h / 6) * (q1 + 2 * q2 + 2 * q3 + q4) for y, q1, q2, q3, q4 in zip(a, d1, d2, d3, d4)]

    def step(self, a, n: int):
        h = self.dz / 2
        a = self._rk4(a, n, 0.0, h)
        a = [np.fft.ifftn(pr * np.fft.fftn(x)) for x, pr in zip(a, self.prop)]
        return self._rk4(a, n, h, h)

    def propagate(self, fields, nsteps: int, n0: int = 0):
        a = [np.array(f, dtype=np.complex128) for f in fields]
        for n in range(n0, n0 + nsteps):
            a = self.step(a, n)
        return a
