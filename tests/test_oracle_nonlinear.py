"""Pins of the oracle's nonlinear half-steps and of the full N/2 - L - N/2
loop (Sec. 3.1) against closed forms, conservation laws, the splitting's
convergence order and the Boyd-Kleinman optimum printed in Sec. 5.2."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import ssfm
from tests.util import bk_efficiency, bk_integral, rel_l2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _uniform(vals, shape=(2, 2, 2)):
    return [torch.full(shape, complex(v), dtype=torch.complex128) for v in vals]


def _fp(**k):
    return ssfm.FieldParams(**k)


# Plane waves: a uniform field only has the k = 0 mode, whose symbol is
# -alpha/2 = 0, so the loop reduces to 2 NZ RK4 steps of the coupled ODEs.

@pytest.mark.parametrize("dk", [0.0, 3.0, -7.5])
def test_undepleted_shg_sinc(dk):
    """kappa_F = 0: S(L) = i kappa_S F0^2 int_0^L exp(-i dk z) dz, i.e.
    |S|^2 = kappa_S^2 |F0|^4 L^2 sinc^2(dk L/2)."""
    f0, ks, nz = 0.8 + 0.3j, 1.7, 100
    prob = ssfm.Problem(2, 2, 2, 2, 1.0 / nz, [_fp(kappa=0.0), _fp(kappa=ks)], dk_const=dk)
    f, s = ssfm.propagate(_uniform([f0, 0]), prob, nz)
    integral = 1.0 if dk == 0 else (1 - np.exp(-1j * dk)) / (1j * dk)
    want = 1j * ks * f0 ** 2 * integral
    assert abs(complex(s[0, 0, 0]) - want) / abs(want) < 1e-9
    assert abs(complex(f[0, 0, 0]) - f0) < 1e-15
    sinc = 1.0 if dk == 0 else math.sin(dk / 2) / (dk / 2)
    assert abs(abs(complex(s[0, 0, 0])) ** 2 - ks ** 2 * abs(f0) ** 4 * sinc ** 2) < 1e-9


def test_depleted_shg_sech_tanh():
    """dk = 0: F = F0 sech(G z), S = i sqrt(kS/kF) F0 tanh(G z), G = sqrt(kF kS) F0."""
    kf, ks, f0, nz = 1.3, 0.6, 1.5, 100
    prob = ssfm.Problem(2, 2, 2, 2, 1.0 / nz, [_fp(kappa=kf), _fp(kappa=ks)])
    f, s = ssfm.propagate(_uniform([f0, 0]), prob, nz)
    g = math.sqrt(kf * ks) * f0
    assert abs(complex(f[0, 0, 0]) - f0 / math.cosh(g)) < 1e-9
    assert abs(complex(s[0, 0, 0]) - 1j * math.sqrt(ks / kf) * f0 * math.tanh(g)) < 1e-9


def test_opa_cosh_sinh():
    """kappa_p = 0, dk = 0: A_s = A_s0 cosh(g z), A_i = i k_i A_p A_s0* sinh(g z)/g,
    g = sqrt(k_s k_i) |A_p|."""
    ap, as0, ks, ki, nz = 1.2 * np.exp(0.4j), 0.01 - 0.02j, 1.5, 0.9, 100
    prob = ssfm.Problem(2, 2, 2, 3, 1.0 / nz, [_fp(kappa=0.0), _fp(kappa=ks), _fp(kappa=ki)])
    p, s, i = ssfm.propagate(_uniform([ap, as0, 0]), prob, nz)
    g = math.sqrt(ks * ki) * abs(ap)
    want_s = as0 * math.cosh(g)
    want_i = 1j * ki * ap * np.conj(as0) * math.sinh(g) / g
    assert abs(complex(s[0, 0, 0]) - want_s) / abs(want_s) < 1e-9
    assert abs(complex(i[0, 0, 0]) - want_i) / abs(want_i) < 1e-9
    assert abs(complex(p[0, 0, 0]) - ap) < 1e-15


@pytest.mark.parametrize("dk", [0.0, 4.0])
def test_undepleted_sfg(dk):
    """kappa_s = kappa_i = 0: A_p(L) = i k_p A_s A_i int_0^L exp(-i dk z) dz."""
    a_s, a_i, kp, nz = 0.7 + 0.1j, -0.4 + 0.9j, 2.2, 100
    prob = ssfm.Problem(2, 2, 2, 3, 1.0 / nz, [_fp(kappa=kp), _fp(), _fp()], dk_const=dk)
    p, s, i = ssfm.propagate(_uniform([0, a_s, a_i]), prob, nz)
    integral = 1.0 if dk == 0 else (1 - np.exp(-1j * dk)) / (1j * dk)
    want = 1j * kp * a_s * a_i * integral
    assert abs(complex(p[0, 0, 0]) - want) / abs(want) < 1e-9


def test_step_profile_phase_closed_form():
    """Per-step dk_n: Phi is the integral of the piecewise-constant profile, so
    for undepleted SHG S(L) = i kS F0^2 sum_n exp(-i Phi_n)(1 - exp(-i dk_n dz))/(i dk_n)."""
    nz, ks, f0 = 50, 1.0, 1.0
    rng = np.random.default_rng(11)
    dks = rng.uniform(-8, 8, nz)
    dz = 1.0 / nz
    prob = ssfm.Problem(2, 2, 2, 2, dz, [_fp(kappa=0.0), _fp(kappa=ks)], dk=list(dks))
    f, s = ssfm.propagate(_uniform([f0, 0]), prob, nz)
    phi = np.concatenate([[0.0], np.cumsum(dks * dz)])
    want = 1j * ks * f0 ** 2 * sum(np.exp(-1j * phi[n]) * (1 - np.exp(-1j * dks[n] * dz)) / (1j * dks[n])
                                   for n in range(nz))
    assert abs(complex(s[0, 0, 0]) - want) / abs(want) < 1e-8


def test_constant_profile_equals_constant_dk():
    rng = np.random.default_rng(12)
    a = [torch.from_numpy(rng.standard_normal((4, 4, 4)) + 1j * rng.standard_normal((4, 4, 4)))
         for _ in range(3)]
    fps = [_fp(kappa=1.0, diffraction=0.5, k2=0.3), _fp(kappa=0.8, tan_rho=0.2),
           _fp(kappa=0.6, delay=0.4)]
    p1 = ssfm.Problem(4, 4, 4, 3, 0.05, fps, dk_const=2.5)
    p2 = ssfm.Problem(4, 4, 4, 3, 0.05, fps, dk=[2.5] * 20)
    o1 = ssfm.propagate(a, p1, 20)
    o2 = ssfm.propagate(a, p2, 20)
    for x, y in zip(o1, o2):
        assert rel_l2(x.numpy(), y.numpy()) < 1e-12


def _random_smooth(rng, nf, n, amp):
    x = ssfm.axis_coords(n).numpy()
    env = np.exp(-(x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2) / (n / 3) ** 2)
    return [torch.from_numpy(amp * env * (rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))))
            for _ in range(nf)]


def _mr_drift(nf, nz, dk):
    rng = np.random.default_rng(21)
    a = _random_smooth(rng, nf, 8, 0.6)
    if nf == 3:
        fps = [_fp(kappa=1.1, diffraction=0.3, tan_rho=0.2, k2=0.5), _fp(kappa=0.8, diffraction=0.4, delay=0.3),
               _fp(kappa=0.5, diffraction=0.7, k2=-0.4, k3=0.1)]
    else:
        fps = [_fp(kappa=1.1, diffraction=0.3, k2=0.5), _fp(kappa=0.7, diffraction=0.15, tan_rho=0.3)]
    prob = ssfm.Problem(8, 8, 8, nf, 1.0 / nz, fps, dk_const=dk)
    m0 = np.array(ssfm.manley_rowe(a, prob))
    m1 = np.array(ssfm.manley_rowe(ssfm.propagate(a, prob, nz), prob))
    return np.abs(m1 - m0).max() / np.abs(m0).max()


@pytest.mark.parametrize("nf", [2, 3])
def test_manley_rowe_drift_fourth_order(nf):
    """The linear step conserves each field's energy (alpha = 0) and the
    lossless chi(2) equations conserve the Manley-Rowe combinations, so the
    only drift is the RK4 error, O(dz^4) globally."""
    d1 = _mr_drift(nf, 10, 1.7)
    d2 = _mr_drift(nf, 20, 1.7)
    assert d1 < 1e-4
    assert 12.0 < d1 / d2 < 20.0


def test_global_second_order_convergence():
    """Strang splitting (eq. expon) with RK4 half-steps: global error O(dz^2),
    so successive differences shrink by ~4 per halving of dz."""
    rng = np.random.default_rng(22)
    a = _random_smooth(rng, 3, 8, 1.0)
    fps = [_fp(kappa=1.2, diffraction=0.5, tan_rho=0.3, k2=0.6), _fp(kappa=0.9, diffraction=0.6, delay=0.5),
           _fp(kappa=0.7, diffraction=0.9, k2=-0.5)]
    outs = []
    for nz in (16, 32, 64):
        prob = ssfm.Problem(8, 8, 8, 3, 1.0 / nz, fps, dk_const=2.0)
        outs.append(np.concatenate([x.numpy().ravel() for x in ssfm.propagate(a, prob, nz)]))
    r = np.linalg.norm(outs[0] - outs[1]) / np.linalg.norm(outs[1] - outs[2])
    assert 3.6 < r < 4.4


def _bk_run(xi, dkl, n=128, nz=200, w_focus=None):
    """Undepleted CW SHG of a beam focused at L/2 (Sec. 5.2 set-up):
    returns (SSFM efficiency E_S/P_F^2, closed form kS^2 L |I|^2/(8 pi D_F xi))."""
    dfun = 36.0
    w0 = math.sqrt(2 * dfun / xi)       # zR = w0^2/(4 D) = L/(2 xi)
    x = ssfm.axis_coords(n).numpy()
    r2 = x[None, None, :] ** 2 + x[None, :, None] ** 2
    f0 = 1 / (1 - 1j * xi) * np.exp(-r2 / (w0 ** 2 * (1 - 1j * xi)))
    ks = 1.0
    prob = ssfm.Problem(n, n, 1, 2, 1.0 / nz, [_fp(kappa=0.0, diffraction=dfun),
                                              _fp(kappa=ks, diffraction=dfun / 2)], dk_const=dkl)
    f, s = ssfm.propagate([torch.from_numpy(f0), torch.zeros(1, n, n, dtype=torch.complex128)], prob, nz)
    pf = float((np.abs(f0) ** 2).sum())
    es = float((s.abs() ** 2).sum())
    return es / pf ** 2, bk_efficiency(xi, dkl, dfun, ks)


def test_boyd_kleinman_optimum():
    """Sec. 5.2: focused-beam SHG efficiency agrees with Boyd-Kleinman within
    0.2 % and, at dk = -3.2/L, peaks at xi = 2.84 (values printed there)."""
    with open(os.path.join(GOLDEN, "boyd_kleinman.json")) as fh:
        g = json.load(fh)
    xis = [2.0, g["xi_opt"], 4.0]
    effs = []
    for xi in xis:
        num, closed = _bk_run(xi, g["dk_L"])
        assert abs(num - closed) / closed < g["rel_err_bound"]
        assert abs(num - closed) / closed < 2e-4   # wrap-free grid, NZ = 200
        effs.append(num)
    assert effs[1] > effs[0] and effs[1] > effs[2]
    # the closed form itself peaks there too (BK's h_m ~ 1.068)
    grid = np.linspace(2.0, 4.0, 201)
    h = [abs(bk_integral(-g["dk_L"] / (2 * x), x)) ** 2 / (4 * x) for x in grid]
    assert abs(grid[int(np.argmax(h))] - g["xi_opt"]) < 0.05
    assert abs(max(h) - 1.068) < 2e-3


def test_uniform_transverse_map_equals_shifted_constant_mismatch():
    """dk(x, y, z) = dk + c everywhere is the scalar case with dk + c."""
    rng = np.random.default_rng(41)
    a = _random_smooth(rng, 2, 8, 0.8)
    fps = [_fp(kappa=1.1, diffraction=0.5, tan_rho=0.2, k2=0.4), _fp(kappa=0.8, diffraction=0.25, delay=0.3)]
    nz = 12
    plain = ssfm.propagate(a, ssfm.Problem(8, 8, 8, 2, 1.0 / nz, fps, dk_const=2.5 + 1.25), nz)
    mapped = ssfm.propagate(a, ssfm.Problem(8, 8, 8, 2, 1.0 / nz, fps, dk_const=2.5,
                                            dk_map=np.full((8, 8), 1.25)), nz)
    for x, y in zip(plain, mapped):
        assert float((x - y).abs().max()) < 1e-13 * float(x.abs().max())


def test_transverse_map_undepleted_shg_closed_form():
    """kappa_F = 0 and no linear terms: every (x, y) column is an independent
    undepleted SHG problem with its own mismatch dk + s_n m(x, y), so
    S(L) = i kS F0^2 sum_n exp(-i Phi_n) (1 - exp(-i K_n dz)) / (i K_n) with
    K_n = dk + s_n m and Phi_n = dk z_n + m sum_{l<n} s_l dz.  The map is
    asymmetric in x and y, so a transposed map fails."""
    nx, ny, nt, nz = 5, 3, 2, 100
    rng = np.random.default_rng(42)
    m = rng.uniform(-8, 8, (ny, nx))
    s = rng.uniform(0.2, 1.5, nz)
    dk, ks, f0 = 1.7, 1.3, 0.9 - 0.2j
    fps = [_fp(kappa=0.0), _fp(kappa=ks)]
    prob = ssfm.Problem(nx, ny, nt, 2, 1.0 / nz, fps, dk_const=dk, dk_map=m, dk_map_scale=list(s))
    a0 = [torch.full((nt, ny, nx), f0, dtype=torch.complex128), torch.zeros(nt, ny, nx, dtype=torch.complex128)]
    out = ssfm.propagate(a0, prob, nz)
    dz = 1.0 / nz
    psi = np.concatenate([[0.0], np.cumsum(s * dz)])
    want = np.zeros((ny, nx), complex)
    for n in range(nz):
        k = dk + s[n] * m
        phi_n = dk * n * dz + m * psi[n]
        want += np.exp(-1j * phi_n) * (1 - np.exp(-1j * k * dz)) / (1j * k)
    want *= 1j * ks * f0 ** 2
    got = out[1].numpy()
    assert np.abs(got - want[None]).max() < 1e-9 * np.abs(want).max()
    assert np.abs(out[0].numpy() - f0).max() < 1e-13   # F is not driven (kappa_F = 0)
