"""Seeded synthetic inputs: entrance fields and the parameter sets of the
benchmark workloads.

This module only builds inputs.  It holds none of the propagation arithmetic,
and both the engine's tests and the oracle consume what it produces.  Every
field is generated in float64 and rounded once to complex64; the oracle is
given those rounded values, so input rounding is never part of a parity error.

Field shapes are [nt, ny, nx] (x fastest).  Grid coordinates are centred,
x_a = (a - floor(n/2)) in cells; z is measured in crystal lengths L = 1.

Entrance field (eq. gaussianbeamc with the Gaussian pulse envelope of the
illustrative example, Sec. 6):
    A(x, y, tau) = A0/(1 - i xi) exp[-(x^2 + y^2)/(w0^2 (1 - i xi)) - (tau/tau0)^2]
with xi = L/(2 z_R) the focusing parameter and z_R = w0^2/(4 D) in the
normalised units (D = 1/(2k)), so the beam focuses at z = L/2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# omega_p : omega_s : omega_i of the paper's OPG example (1064, 1450, 3997 nm)
OMEGA_RATIO = (1.0, 1064.0 / 1450.0, 1064.0 / 3997.0)


def fwhm_to_tau0(fwhm: float) -> float:
    """Intensity FWHM of exp(-2 (tau/tau0)^2) -> tau0."""
    return fwhm / math.sqrt(2.0 * math.log(2.0))


def centred(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) - (n // 2)


def focused_pulse(nx: int, ny: int, nt: int, w0: float, tau0: Optional[float],
                  xi: float, a0: float = 1.0) -> np.ndarray:
    """complex128 entrance field of a beam focused at L/2 (see module doc).
    tau0=None gives a CW field (constant in tau)."""
    x = centred(nx)[None, None, :]
    y = centred(ny)[None, :, None]
    t = centred(nt)[:, None, None]
    q = 1.0 - 1j * xi
    spatial = a0 / q * np.exp(-(x ** 2 + y ** 2) / (w0 ** 2 * q))
    if tau0 is None:
        temporal = np.ones_like(t)
    else:
        temporal = np.exp(-(t / tau0) ** 2)
    return spatial * temporal


def to_c64(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a.astype(np.complex64))


@dataclass
class FieldSpec:
    kappa: float = 0.0
    diffraction: float = 0.0
    tan_rho: float = 0.0
    delay: float = 0.0
    k2: float = 0.0
    k3: float = 0.0
    alpha: float = 0.0


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nt: int
    nf: int
    nz: int
    dz: float
    fields: List[FieldSpec]
    dk_const: float = 0.0
    dk: Optional[np.ndarray] = None
    init: List[np.ndarray] = field(default_factory=list)  # complex64 arrays
    # transverse mismatch map: dk(x, y, z) = dk_n + s_n dk_map[y, x] in step n
    dk_map: Optional[np.ndarray] = None
    dk_map_scale: Optional[np.ndarray] = None

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nt


def shg32(seed: int = 1, nz: int = 100, with_fields: bool = True) -> Workload:
    """SHG, 2 fields, 32^3, 100 steps: w0 = 8 cells, pulse FWHM 6 cells,
    xi = 0.5, dk = 0.5/L, SH walk-off 0.1 cell/step, GVD of opposite sign
    per field (dispersion length L), kappa = 1 (nonlinear length ~ L)."""
    n = 32
    w0, tau0, xi = 8.0, fwhm_to_tau0(6.0), 0.5
    d_f = xi * w0 ** 2 / 2.0
    k2 = tau0 ** 2 / 2.0
    dz = 1.0 / nz
    fs = [FieldSpec(kappa=1.0, diffraction=d_f, k2=+k2),
          FieldSpec(kappa=1.0, diffraction=d_f / 2.0, tan_rho=0.1 / 0.01, k2=-k2)]
    wl = Workload("shg32", n, n, n, 2, nz, dz, fs, dk_const=0.5)
    if with_fields:
        f = focused_pulse(n, n, n, w0, tau0, xi)
        wl.init = [to_c64(f), np.zeros((n, n, n), np.complex64)]
    return wl


def sfg128(seed: int = 2, n: int = 128, nz: int = 500,
           with_fields: bool = True) -> Workload:
    """SFG, 3 fields, 128^3, 500 steps: s and i are focused Gaussian pulses
    (w0 = 20 and 24 cells, FWHM 16 and 20 cells) with seeded 0-0.1 rad
    spatial phase noise, p starts at zero; dk = 3/L, p walk-off 0.05
    cell/step, distinct group delays and GVD, nonlinear length 0.2 L."""
    om = OMEGA_RATIO
    w_s, w_i = 20.0, 24.0
    t_s, t_i = fwhm_to_tau0(16.0), fwhm_to_tau0(20.0)
    d_s = 100.0
    d = [d_s * om[1] / om[0], d_s, d_s * om[1] / om[2]]
    k0 = 5.0 / math.sqrt(om[0] * om[1])
    kap = [k0 * om[0], k0 * om[1], k0 * om[2]]
    dz = 1.0 / nz
    k2 = [50.0, 92.33, -144.27]
    delay = [8.0, 0.0, -6.0]
    fs = [FieldSpec(kappa=kap[j], diffraction=d[j], delay=delay[j], k2=k2[j])
          for j in range(3)]
    fs[0].tan_rho = 0.05 / 0.002
    wl = Workload("sfg128", n, n, n, 3, nz, dz, fs, dk_const=3.0)
    if with_fields:
        rng = np.random.default_rng(seed)
        xi_s = 2.0 * d[1] / w_s ** 2
        xi_i = 2.0 * d[2] / w_i ** 2
        scr_s = np.exp(1j * rng.uniform(0.0, 0.1, size=(n, n)))[None]
        scr_i = np.exp(1j * rng.uniform(0.0, 0.1, size=(n, n)))[None]
        s = focused_pulse(n, n, n, w_s, t_s, xi_s) * scr_s
        i = focused_pulse(n, n, n, w_i, t_i, xi_i) * scr_i
        wl.init = [np.zeros((n, n, n), np.complex64), to_c64(s), to_c64(i)]
    return wl


def opg256(seed: int = 3, n: int = 256, nz: int = 1000,
           with_fields: bool = True) -> Workload:
    """OPG, 3 fields, 256^3, 1000 steps: strong focused pump (w0 = 40,
    FWHM 48 cells, xi = 0.5), signal and idler seeded with complex Gaussian
    noise of rms 1e-6 of the pump amplitude; dk = 0; walk-off, group delay
    and GVD on every field; parametric gain 10/L."""
    om = OMEGA_RATIO
    w_p, t_p, xi_p = 40.0, fwhm_to_tau0(48.0), 0.5
    d_p = xi_p * w_p ** 2 / 2.0
    d = [d_p, d_p * om[0] / om[1], d_p * om[0] / om[2]]
    k0 = 10.0 / math.sqrt(om[1] * om[2])
    kap = [k0 * om[0], k0 * om[1], k0 * om[2]]
    dz = 1.0 / nz
    tr = [20.0, 10.0, -10.0]
    delay = [12.0, 0.0, -16.0]
    k2 = [831.0, 600.0, -900.0]
    fs = [FieldSpec(kappa=kap[j], diffraction=d[j], tan_rho=tr[j],
                    delay=delay[j], k2=k2[j]) for j in range(3)]
    wl = Workload("opg256", n, n, n, 3, nz, dz, fs, dk_const=0.0)
    if with_fields:
        rng = np.random.default_rng(seed)
        p = focused_pulse(n, n, n, w_p, t_p, xi_p)
        sig = 1e-6 * math.sqrt(0.5)
        s = sig * (rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n)))
        i = sig * (rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n)))
        wl.init = [to_c64(p), to_c64(s), to_c64(i)]
    return wl


SWEEP_SHAPES = [(64, 64, 64), (96, 96, 64), (128, 128, 64), (128, 128, 256)]


def shg_sweep_instance(rng: np.random.Generator, with_fields: bool = True,
                       shape=None, nz=None) -> Workload:
    """One instance of the batched SHG sweep: grid drawn from SWEEP_SHAPES,
    dk L uniform in [-6, 6], focusing parameter log-uniform in [0.1, 10],
    200-600 steps; w0 = nx/8, FWHM = nt/8, SH walk-off nx/16 cells/L."""
    if shape is None:
        shape = SWEEP_SHAPES[int(rng.integers(0, len(SWEEP_SHAPES)))]
    nx, ny, nt = shape
    dkl = float(rng.uniform(-6.0, 6.0))
    xi = float(math.exp(rng.uniform(math.log(0.1), math.log(10.0))))
    nzi = int(rng.integers(200, 601)) if nz is None else nz
    w0 = nx / 8.0
    tau0 = fwhm_to_tau0(nt / 8.0)
    d_f = xi * w0 ** 2 / 2.0
    k2 = tau0 ** 2 / 2.0
    fs = [FieldSpec(kappa=1.0, diffraction=d_f, k2=+k2),
          FieldSpec(kappa=1.0, diffraction=d_f / 2.0, tan_rho=nx / 16.0, k2=-k2)]
    wl = Workload(f"shg{nx}x{ny}x{nt}", nx, ny, nt, 2, nzi, 1.0 / nzi, fs,
                  dk_const=dkl)
    if with_fields:
        f = focused_pulse(nx, ny, nt, w0, tau0, xi)
        wl.init = [to_c64(f), np.zeros((nt, ny, nx), np.complex64)]
    return wl


def shg_sweep(seed: int = 4, count: int = 64, with_fields: bool = True) -> List[Workload]:
    rng = np.random.default_rng(seed)
    return [shg_sweep_instance(rng, with_fields) for _ in range(count)]


def shg_adjoint(seed: int = 5, with_fields: bool = True) -> Workload:
    """Inverse-design SHG: 128 x 128 x 64, 400 steps, w0 = 16, FWHM 8,
    xi = 1, GVD of opposite sign, no walk-off; per-step dk_n = 2/L plus
    seeded N(0, 0.1/L) noise."""
    nx, ny, nt, nz = 128, 128, 64, 400
    w0, tau0, xi = 16.0, fwhm_to_tau0(8.0), 1.0
    d_f = xi * w0 ** 2 / 2.0
    k2 = tau0 ** 2 / 2.0
    fs = [FieldSpec(kappa=1.0, diffraction=d_f, k2=+k2),
          FieldSpec(kappa=1.0, diffraction=d_f / 2.0, k2=-k2)]
    rng = np.random.default_rng(seed)
    dk = 2.0 + 0.1 * rng.standard_normal(nz)
    wl = Workload("shg_adjoint", nx, ny, nt, 2, nz, 1.0 / nz, fs, dk=dk)
    if with_fields:
        f = focused_pulse(nx, ny, nt, w0, tau0, xi)
        wl.init = [to_c64(f), np.zeros((nt, ny, nx), np.complex64)]
    return wl


def random_fields(rng: np.random.Generator, nf: int, nx: int, ny: int, nt: int,
                  scale: float = 1.0, smooth: Optional[float] = None) -> List[np.ndarray]:
    """Seeded complex Gaussian fields (optionally multiplied by a broad
    Gaussian envelope of 1/e radius `smooth` cells) for parity cases."""
    out = []
    for _ in range(nf):
        a = rng.standard_normal((nt, ny, nx)) + 1j * rng.standard_normal((nt, ny, nx))
        a *= scale / math.sqrt(2.0)
        if smooth is not None:
            x = centred(nx)[None, None, :]
            y = centred(ny)[None, :, None]
            t = centred(nt)[:, None, None]
            a = a * np.exp(-(x ** 2 + y ** 2 + t ** 2) / smooth ** 2)
        out.append(to_c64(a))
    return out


# ---------------------------------------------------------------------------
# Reduced-dimension workloads (CW beams with nt = 1, plane-wave pulses with
# nx = ny = 1), run as batches.
# ---------------------------------------------------------------------------
BK_DIFFRACTION = 36.0   # D_F of the CW focusing sweep (cells^2 / L)
BK_XI = tuple(round(2.0 + 0.2 * k, 3) for k in range(11))       # 2.0 .. 4.0
BK_DKL = tuple(round(-4.0 + 0.2 * k, 3) for k in range(9))      # -4.0 .. -2.4


def bk_cw_instance(xi: float, dkl: float, n: int = 128, nz: int = 200) -> Workload:
    """Undepleted CW SHG of a beam focused at L/2 (the focusing study of
    Sec. 5.2): nt = 1, kappa_F = 0, kappa_S = 1, D_S = D_F / 2, no walk-off;
    w0 from xi = L / (2 z_R) with z_R = w0^2 / (4 D_F)."""
    w0 = math.sqrt(2.0 * BK_DIFFRACTION / xi)
    fs = [FieldSpec(kappa=0.0, diffraction=BK_DIFFRACTION),
          FieldSpec(kappa=1.0, diffraction=BK_DIFFRACTION / 2.0)]
    wl = Workload(f"bk_xi{xi}_dk{dkl}", n, n, 1, 2, nz, 1.0 / nz, fs, dk_const=dkl)
    wl.init = [to_c64(focused_pulse(n, n, 1, w0, None, xi)), np.zeros((1, n, n), np.complex64)]
    return wl


def bk_sweep(n: int = 128, nz: int = 200) -> List[Workload]:
    """The focusing-parameter x phase-mismatch grid BK_XI x BK_DKL (99 CW
    problems), xi-major."""
    return [bk_cw_instance(xi, dkl, n, nz) for xi in BK_XI for dkl in BK_DKL]


def plane_wave_pulse_sweep(seed: int = 6, count: int = 16, nt: int = 256) -> List[Workload]:
    """Pulsed plane-wave SHG (nx = ny = 1): Gaussian F pulse of FWHM nt/8,
    group-velocity mismatch delta_S in U[-nt/8, nt/8] cells/L, GVD k''_F =
    +tau0^2/2 and k''_S = -tau0^2/2 (dispersion length L), dk L in U[-6, 6],
    kappa = 1 with peak amplitude in U[0.5, 2] (pump depletion), 100-300
    steps."""
    rng = np.random.default_rng(seed)
    tau0 = fwhm_to_tau0(nt / 8.0)
    out = []
    for k in range(count):
        amp = float(rng.uniform(0.5, 2.0))
        fs = [FieldSpec(kappa=1.0, k2=tau0 ** 2 / 2.0),
              FieldSpec(kappa=1.0, delay=float(rng.uniform(-nt / 8.0, nt / 8.0)), k2=-tau0 ** 2 / 2.0)]
        nzk = int(rng.integers(100, 301))
        wl = Workload(f"pw{k}", 1, 1, nt, 2, nzk, 1.0 / nzk, fs, dk_const=float(rng.uniform(-6.0, 6.0)))
        wl.init = [to_c64(focused_pulse(1, 1, nt, 1.0, tau0, 0.0, amp)),
                   np.zeros((nt, 1, 1), np.complex64)]
        out.append(wl)
    return out


def shg_thermal(seed: int = 7, with_fields: bool = True) -> Workload:
    """SHG through a crystal with a transverse mismatch map (thermal dephasing
    plus poling nonuniformity): 128 x 128 x 64, 200 steps, w0 = 16, FWHM 8,
    xi = 1, dk_0 = 1/L; m(x, y) = -3 exp(-2 r^2 / (2 w0)^2) + U[-0.25, 0.25]
    per transverse cell (seeded); s_n = 1 - z_n / 2 (the heat load decays
    along the crystal)."""
    nx, ny, nt, nz = 128, 128, 64, 200
    w0, tau0, xi = 16.0, fwhm_to_tau0(8.0), 1.0
    d_f = xi * w0 ** 2 / 2.0
    k2 = tau0 ** 2 / 2.0
    fs = [FieldSpec(kappa=1.0, diffraction=d_f, k2=+k2),
          FieldSpec(kappa=1.0, diffraction=d_f / 2.0, k2=-k2)]
    rng = np.random.default_rng(seed)
    x = centred(nx)[None, :]
    y = centred(ny)[:, None]
    m = -3.0 * np.exp(-2.0 * (x ** 2 + y ** 2) / (2.0 * w0) ** 2) + rng.uniform(-0.25, 0.25, (ny, nx))
    dz = 1.0 / nz
    scale = 1.0 - 0.5 * dz * np.arange(nz)
    wl = Workload("shg_thermal", nx, ny, nt, 2, nz, dz, fs, dk_const=1.0, dk_map=m, dk_map_scale=scale)
    if with_fields:
        f = focused_pulse(nx, ny, nt, w0, tau0, xi)
        wl.init = [to_c64(f), np.zeros((nt, ny, nx), np.complex64)]
    return wl
