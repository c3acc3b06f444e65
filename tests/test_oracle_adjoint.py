"""Pins of the oracle's adjoint (oracle/adjoint.py): central finite
differences in FP64 (h = 1e-3), the closed-form gradient of undepleted
plane-wave SHG with a per-step mismatch profile, and, without coupling,
the adjoint of the unitary linear propagation being backward propagation."""
import math

import numpy as np
import torch

from oracle import adjoint, ssfm


def _problem(nz=12, n=8, nt=4):
    fps = [ssfm.FieldParams(kappa=1.1, diffraction=0.6, tan_rho=0.2, k2=0.5),
           ssfm.FieldParams(kappa=0.9, diffraction=0.3, delay=0.4, k2=-0.5)]
    rng = np.random.default_rng(31)
    dk = 2.0 + 0.5 * rng.standard_normal(nz)
    prob = ssfm.Problem(n, n, nt, 2, 1.0 / nz, fps, dk=list(dk))
    x = ssfm.axis_coords(n).numpy()
    t = ssfm.axis_coords(nt).numpy()
    env = np.exp(-(x[None, None, :] ** 2 + x[None, :, None] ** 2) / 6.0 - t[:, None, None] ** 2 / 3.0)
    f = env * (1.0 + 0.3 * (rng.standard_normal(env.shape) + 1j * rng.standard_normal(env.shape)))
    s = 0.2 * env * (rng.standard_normal(env.shape) + 1j * rng.standard_normal(env.shape))
    return prob, [torch.from_numpy(f), torch.from_numpy(s)], dk


def test_dk_gradient_matches_central_differences():
    prob, a0, dk = _problem()
    nz = len(dk)
    j, g_fields, g_dk = adjoint.gradients(a0, dk, prob, nz)
    h = 1e-3
    for n in range(nz):
        dp, dm = dk.copy(), dk.copy()
        dp[n] += h
        dm[n] -= h
        fd = (adjoint.loss_value(a0, dp, prob, nz) - adjoint.loss_value(a0, dm, prob, nz)) / (2 * h)
        assert abs(fd - float(g_dk[n])) <= 1e-5 * max(abs(fd), 1e-3 * abs(j)), (n, fd, float(g_dk[n]))


def test_field_gradient_matches_central_differences():
    """Directional derivative along random complex directions v with
    ||v|| = ||A_in||: dJ = sum Re(conj(g) v) in PyTorch's convention."""
    prob, a0, dk = _problem()
    nz = len(dk)
    j, g_fields, _ = adjoint.gradients(a0, dk, prob, nz)
    rng = np.random.default_rng(5)
    norm = math.sqrt(sum(float((x.abs() ** 2).sum()) for x in a0))

    def fd(v, h):
        jp = adjoint.loss_value([x + h * y for x, y in zip(a0, v)], dk, prob, nz)
        jm = adjoint.loss_value([x - h * y for x, y in zip(a0, v)], dk, prob, nz)
        return (jp - jm) / (2 * h)

    for _ in range(4):
        v = [torch.from_numpy(rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)) for x in a0]
        vn = math.sqrt(sum(float((x.abs() ** 2).sum()) for x in v))
        v = [x * (norm / vn) for x in v]
        an = sum(float((torch.conj(g) * y).real.sum()) for g, y in zip(g_fields, v))
        e1 = abs(fd(v, 1e-3) - an)
        e2 = abs(fd(v, 5e-4) - an)
        assert e1 <= 1e-5 * abs(an), (e1, an)
        # the discrepancy is the O(h^2) truncation of the difference quotient
        assert 3.0 < e1 / e2 < 5.0, (e1, e2)


def test_closed_form_plane_wave_gradient():
    """kappa_F = 0, uniform F0: S(L) = i kS F0^2 sum_n exp(-i Phi_n)(1 - exp(-i dk_n dz))/(i dk_n)
    (exact solution of the ODE).  J = -M |S(L)|^2 over M grid points, so
    dJ/ddk_n and dJ/dF0 follow by differentiating this expression."""
    nz, ks = 40, 1.3
    rng = np.random.default_rng(8)
    dks = rng.uniform(-6, 6, nz)
    f0 = 0.7 - 0.4j
    shape = (2, 2, 2)
    m = int(np.prod(shape))
    prob = ssfm.Problem(2, 2, 2, 2, 1.0 / nz, [ssfm.FieldParams(kappa=0.0), ssfm.FieldParams(kappa=ks)],
                        dk=list(dks))
    a0 = [torch.full(shape, f0, dtype=torch.complex128), torch.zeros(shape, dtype=torch.complex128)]
    _, g_fields, g_dk = adjoint.gradients(a0, dks, prob, nz)

    d = torch.tensor(dks, dtype=torch.float64, requires_grad=True)
    fr = torch.tensor([f0.real, f0.imag], dtype=torch.float64, requires_grad=True)
    F = torch.complex(fr[0], fr[1])
    dz = 1.0 / nz
    phi = torch.cat([d.new_zeros(1), torch.cumsum(d * dz, 0)])[:-1]
    seg = torch.exp(-1j * phi) * (1 - torch.exp(-1j * d * dz)) / (1j * d)
    S = 1j * ks * F ** 2 * seg.sum()
    J = -m * S.abs() ** 2
    gd, gf = torch.autograd.grad(J, [d, fr])
    # what remains is the O(h^4) error of RK4 against the exact ODE solution
    # (4.5e-8 at 40 steps, 6.9e-7 at 20)
    assert float((g_dk - gd).abs().max()) < 2e-7 * float(gd.abs().max())
    # every grid point carries the same field, so each gets 1/m of dJ/dF0
    want = complex(float(gf[0]), float(gf[1])) / m
    got = g_fields[0].reshape(-1)
    assert float((got - want).abs().max()) < 1e-7 * abs(want)


def test_uncoupled_adjoint_is_backward_propagation():
    """kappa = 0 and alpha = 0: A(L) = U A(0) with U unitary (Sec. 3.1's
    linear operator only), so for J = Re sum conj(w) A(L) the gradient
    dJ/dRe A(0) + i dJ/dIm A(0) is U^H w = U^-1 w, i.e. w propagated back
    over the same distance (the same loop with dz -> -dz)."""
    nz, n, nt = 10, 8, 8
    fps = [ssfm.FieldParams(kappa=0.0, diffraction=0.7, tan_rho=0.3, delay=-0.4, k2=0.8, k3=0.2),
           ssfm.FieldParams(kappa=0.0, diffraction=0.35, tan_rho=-0.2, delay=0.5, k2=-0.6)]
    rng = np.random.default_rng(17)
    shape = (nt, n, n)
    a0 = [torch.from_numpy(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) for _ in fps]
    w = [torch.from_numpy(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) for _ in fps]
    prob = ssfm.Problem(n, n, nt, 2, 1.0 / nz, fps, dk_const=1.5)

    def loss(out, p):
        return sum((torch.conj(wj) * oj).real.sum() for wj, oj in zip(w, out))

    _, g, g_dk = adjoint.gradients(a0, [1.5] * nz, prob, nz, loss=loss)
    back = ssfm.Problem(n, n, nt, 2, -1.0 / nz, fps, dk_const=1.5)
    want = ssfm.propagate(w, back, nz)
    for gj, wj in zip(g, want):
        assert float((gj - wj).abs().max()) < 1e-12 * float(wj.abs().max())
    assert float(g_dk.abs().max()) == 0.0   # no coupling, no dependence on dk
