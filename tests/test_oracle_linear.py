"""Pins of the oracle's linear step (eqs. dispOp, diffOp; Sec. 3.1 Fourier
step) against things other than itself: brute-force DFTs, symbolic
derivatives of analytic fields, and closed-form solutions."""
import math

import numpy as np
import pytest
import sympy as sp
import torch

from oracle import ssfm
from tests.util import rel_l2


def _prob(nx, ny, nt, **fp):
    return ssfm.Problem(nx, ny, nt, 2, 0.01, [ssfm.FieldParams(**fp), ssfm.FieldParams()])


def _dft_matrix(n, sign):
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


@pytest.mark.parametrize("shape", [(3, 6, 4), (2, 5, 3), (4, 4, 8), (9, 18, 4), (2, 36, 9)])
def test_linear_step_matches_bruteforce_dft(shape):
    """exp(L dz) = F^-1 diag(exp(Lambda dz)) F with F the plain O(n^2) DFT
    along each axis (forward sign -, inverse normalised by 1/n)."""
    nt, ny, nx = shape
    prob = _prob(nx, ny, nt, diffraction=0.7, tan_rho=0.3, delay=-0.4,
                 k2=0.9, k3=0.35, alpha=0.2)
    rng = np.random.default_rng(7)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    lam = ssfm.linear_symbol(prob.fields[0], prob).numpy()
    fx, fy, ft = (_dft_matrix(n, -1) for n in (nx, ny, nt))
    spec = np.einsum("ka,tya->tyk", fx, a)
    spec = np.einsum("ky,tyx->tkx", fy, spec)
    spec = np.einsum("kt,tyx->kyx", ft, spec)
    spec = spec * np.exp(lam * 0.37)
    bx, by, bt = (_dft_matrix(n, +1) / n for n in (nx, ny, nt))
    out = np.einsum("ak,tyk->tya", bx, spec)
    out = np.einsum("yk,tkx->tyx", by, out)
    out = np.einsum("tk,kyx->tyx", bt, out)
    got = ssfm.linear_step(torch.from_numpy(a), torch.from_numpy(lam), 0.37).numpy()
    assert rel_l2(got, out) < 1e-13


def test_frequency_order_and_nyquist():
    """Bins follow 2 pi fftfreq: 0, 1, ..., then negative; even n puts the
    Nyquist bin at -pi/d; grid is centred at floor(n/2)."""
    w = ssfm.angular_freqs(8, 1.0).numpy()
    assert np.allclose(w, 2 * np.pi * np.array([0, 1, 2, 3, -4, -3, -2, -1]) / 8)
    w = ssfm.angular_freqs(5, 2.0).numpy()
    assert np.allclose(w, 2 * np.pi * np.array([0, 1, 2, -2, -1]) / 10)
    assert np.allclose(ssfm.axis_coords(4).numpy(), [-2, -1, 0, 1])
    assert np.allclose(ssfm.axis_coords(5).numpy(), [-2, -1, 0, 1, 2])


# Symbolic pin: d/dz of the propagated field at z = 0 must equal the linear
# operator of eqs. dispOp/diffOp (readings in the oracle's header) applied to
# an analytic field by exact differentiation.
_X, _Y, _T = sp.symbols("x y t", real=True)
_W = 7.0


def _analytic_field():
    # broad, chirped, tilted Gaussian: every odd and even derivative is nonzero
    return sp.exp(-(_X ** 2 + (_Y - 1) ** 2) / _W ** 2 - (_T + 1) ** 2 / (_W - 1) ** 2
                  + sp.I * (sp.Rational(3, 10) * _X + sp.Rational(1, 5) * _T
                            + sp.Rational(1, 50) * _X * _T))


def _apply_operator(expr, D=0, tr=0, delta=0, k2=0, k3=0, alpha=0):
    I = sp.I
    return (I * D * (sp.diff(expr, _X, 2) + sp.diff(expr, _Y, 2))
            - tr * sp.diff(expr, _X)
            - delta * sp.diff(expr, _T)
            - I * sp.Rational(1, 2) * k2 * sp.diff(expr, _T, 2)
            + sp.Rational(1, 6) * k3 * sp.diff(expr, _T, 3)
            - sp.Rational(1, 2) * alpha * expr)


@pytest.mark.parametrize("coef", [
    dict(D=sp.Rational(3, 2)), dict(tr=sp.Rational(7, 10)), dict(delta=sp.Rational(-9, 10)),
    dict(k2=sp.Rational(13, 10)), dict(k3=sp.Rational(11, 10)), dict(alpha=sp.Rational(2, 5)),
    dict(D=1, tr=sp.Rational(1, 2), delta=sp.Rational(1, 3), k2=-1, k3=sp.Rational(1, 2),
         alpha=sp.Rational(1, 10)),
])
def test_linear_generator_matches_symbolic_operator(coef):
    n = 64
    expr = _analytic_field()
    lexpr = _apply_operator(expr, **coef)
    f = sp.lambdify((_X, _Y, _T), expr, "numpy")
    g = sp.lambdify((_X, _Y, _T), lexpr, "numpy")
    x = ssfm.axis_coords(n).numpy()[None, None, :]
    y = ssfm.axis_coords(n).numpy()[None, :, None]
    t = ssfm.axis_coords(n).numpy()[:, None, None]
    a = np.asarray(f(x, y, t) * np.ones((n, n, n)), dtype=np.complex128)
    la = np.asarray(g(x, y, t) * np.ones((n, n, n)), dtype=np.complex128)
    fp = dict(diffraction=float(coef.get("D", 0)), tan_rho=float(coef.get("tr", 0)),
              delay=float(coef.get("delta", 0)), k2=float(coef.get("k2", 0)),
              k3=float(coef.get("k3", 0)), alpha=float(coef.get("alpha", 0)))
    prob = _prob(n, n, n, **fp)
    lam = ssfm.linear_symbol(prob.fields[0], prob)
    eps = 1e-4
    at = torch.from_numpy(a)
    dadz = (ssfm.linear_step(at, lam, eps) - ssfm.linear_step(at, lam, -eps)).numpy() / (2 * eps)
    assert rel_l2(dadz, la) < 1e-6


def test_gaussian_beam_closed_form():
    """Entrance field of eq. gaussianbeamc propagated by diffraction alone
    follows eq. gaussianbeam: focus at L/2, w(z) = w0 sqrt(1 + ((z-f)/zR)^2)."""
    n, w0, xi = 64, 4.0, 0.5
    D = xi * w0 ** 2 / 2.0            # zR = w0^2/(4D) = 1/(2 xi)
    zr = w0 ** 2 / (4 * D)
    x = ssfm.axis_coords(n).numpy()[None, None, :]
    y = ssfm.axis_coords(n).numpy()[None, :, None]

    def beam(z):
        q = 1 + 1j * (z - 0.5) / zr
        return np.broadcast_to(1 / q * np.exp(-(x ** 2 + y ** 2) / (w0 ** 2 * q)), (1, n, n))

    prob = ssfm.Problem(n, n, 1, 2, 0.25, [ssfm.FieldParams(diffraction=D), ssfm.FieldParams()])
    lam = ssfm.linear_symbol(prob.fields[0], prob)
    a = torch.from_numpy(np.ascontiguousarray(beam(0.0)))
    widths = []
    for k in range(1, 5):
        a = ssfm.linear_step(a, lam, 0.25)
        assert rel_l2(a.numpy(), beam(0.25 * k)) < 1e-10
        inten = np.abs(a.numpy()[0]) ** 2
        widths.append(math.sqrt(2 * (inten * (x[0] ** 2 + y[0] ** 2)).sum() / inten.sum()))
    expect = [w0 * math.sqrt(1 + ((0.25 * k - 0.5) / zr) ** 2) for k in range(1, 5)]
    assert np.allclose(widths, expect, rtol=1e-8)
    assert widths[1] < widths[0] and widths[1] < widths[2]   # waist at z = L/2


def test_dispersed_pulse_closed_form():
    """GVD alone: exp(-(t/t0)^2) -> (1 - 2 i k'' z/t0^2)^-1/2 exp(-t^2/(t0^2 - 2 i k'' z))."""
    n, t0, k2 = 128, 6.0, 9.0
    t = ssfm.axis_coords(n).numpy()
    prob = ssfm.Problem(1, 1, n, 2, 1.0, [ssfm.FieldParams(k2=k2), ssfm.FieldParams()])
    lam = ssfm.linear_symbol(prob.fields[0], prob)
    a = torch.from_numpy(np.exp(-(t / t0) ** 2).astype(np.complex128).reshape(n, 1, 1))
    for z in (0.3, 1.0, 2.5):
        got = ssfm.linear_step(a, lam, z).numpy().ravel()
        want = (1 - 2j * k2 * z / t0 ** 2) ** -0.5 * np.exp(-t ** 2 / (t0 ** 2 - 2j * k2 * z))
        assert rel_l2(got, want) < 1e-12


@pytest.mark.parametrize("tr,delta,z", [(3.0, 0.0, 2.0), (0.0, -5.0, 1.0), (2.0, 4.0, 1.5)])
def test_walkoff_and_group_delay_shift(tr, delta, z):
    """-tan(rho) dx and -delta dtau translate the field by tan(rho) z cells in
    x and delta z cells in tau; integer shifts are exact on the grid."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal((8, 6, 10)) + 1j * rng.standard_normal((8, 6, 10))
    prob = ssfm.Problem(10, 6, 8, 2, 1.0, [ssfm.FieldParams(tan_rho=tr, delay=delta),
                                            ssfm.FieldParams()])
    lam = ssfm.linear_symbol(prob.fields[0], prob)
    got = ssfm.linear_step(torch.from_numpy(a), lam, z).numpy()
    want = np.roll(a, (int(round(delta * z)), int(round(tr * z))), axis=(0, 2))
    assert rel_l2(got, want) < 1e-13


def test_unitary_and_absorption():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((8, 8, 8)) + 1j * rng.standard_normal((8, 8, 8))
    for alpha in (0.0, 0.8):
        prob = ssfm.Problem(8, 8, 8, 2, 1.0, [ssfm.FieldParams(diffraction=2.0, tan_rho=0.3,
                                                                delay=0.7, k2=1.1, k3=0.4,
                                                                alpha=alpha), ssfm.FieldParams()])
        lam = ssfm.linear_symbol(prob.fields[0], prob)
        out = ssfm.linear_step(torch.from_numpy(a), lam, 1.3).numpy()
        ratio = (np.abs(out) ** 2).sum() / (np.abs(a) ** 2).sum()
        assert abs(ratio - math.exp(-alpha * 1.3)) < 1e-13


def test_two_stage_linear_step_equals_3d_multiply():
    """The paper's dispersion-then-diffraction sub-steps equal one 3D
    multiply, because the two operators commute (Sec. 3.1)."""
    rng = np.random.default_rng(5)
    a = torch.from_numpy(rng.standard_normal((6, 8, 10)) + 1j * rng.standard_normal((6, 8, 10)))
    fp = ssfm.FieldParams(diffraction=1.3, tan_rho=0.4, delay=-0.3, k2=0.8, k3=0.2, alpha=0.1)
    prob = ssfm.Problem(10, 8, 6, 2, 1.0, [fp, ssfm.FieldParams()])
    one = ssfm.linear_step(a, ssfm.linear_symbol(fp, prob), 0.9).numpy()
    two = ssfm.linear_step_two_stage(a, fp, prob, 0.9).numpy()
    assert rel_l2(two, one) < 1e-14


def test_power_trace_of_gaussian_pulse_and_energy():
    """P(tau) of a sampled Gaussian beam-pulse exp(-r^2/w^2 - tau^2/tau0^2):
    the transverse sum of exp(-2 r^2/w^2) over unit cells is pi w^2 / 2 to
    exponential accuracy for w >> 1 cell (Poisson summation), so P(tau) =
    (pi w^2 / 2) exp(-2 tau^2 / tau0^2); and sum_tau P dtau is the energy."""
    n, nt, w, tau0 = 64, 32, 6.0, 5.0
    x = ssfm.axis_coords(n)
    t = ssfm.axis_coords(nt)
    a = torch.exp(-(x[None, None, :] ** 2 + x[None, :, None] ** 2) / w ** 2
                  - t[:, None, None] ** 2 / tau0 ** 2).to(torch.complex128)
    prob = ssfm.Problem(n, n, nt, 2, 0.1, [ssfm.FieldParams(), ssfm.FieldParams()])
    p = ssfm.power_traces([a, 2 * a], prob)
    want = math.pi * w ** 2 / 2 * torch.exp(-2 * t ** 2 / tau0 ** 2)
    assert float((p[0] - want).abs().max()) < 1e-12 * float(want.max())
    assert float((p[1] - 4 * want).abs().max()) < 1e-11 * float(want.max())
    e = ssfm.energies([a, 2 * a], prob)
    assert abs(float(p[0].sum()) * prob.dt - e[0]) < 1e-12 * e[0]
