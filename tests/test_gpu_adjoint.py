"""GPU adjoint (hand-written reverse sweep behind torch.autograd) against the
oracle's own adjoint (autograd through the FP64 loop)."""
import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from oracle import ssfm
from paper_2609_08384_amd import autograd, brahms, inputs
from tests.sketch import count_sketch
from tests.util import oracle_problem, rel_l2

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(nf, shape, nz, seed, profile=True):
    nx, ny, nt = shape
    rng = np.random.default_rng(seed)
    base = [dict(kappa=1.2, diffraction=0.9, tan_rho=0.4, delay=-0.3, k2=0.7),
            dict(kappa=0.8, diffraction=0.5, tan_rho=-0.2, delay=0.2, k2=-0.6),
            dict(kappa=0.6, diffraction=1.4, delay=0.5, k2=0.3)]
    fields = [inputs.FieldSpec(**base[j]) for j in range(nf)]
    init = inputs.random_fields(rng, nf, nx, ny, nt, scale=0.8,
                                smooth=min(d for d in shape if d > 1) / 2.5)
    dk = (2.0 + 0.7 * rng.standard_normal(nz)) if profile else None
    wl = inputs.Workload("adj", nx, ny, nt, nf, nz, 1.0 / nz, fields, dk_const=1.7, dk=dk)
    wl.init = init
    return wl


def _loss(out):
    return -(out[-1].abs() ** 2).sum()  # energy of the last field (SH or idler)


def _gpu_grads(wl, every, order=None):
    params = brahms.params_from_workload(wl)
    x = [torch.from_numpy(a).to(DEV).requires_grad_(True) for a in wl.init]
    dk = None if wl.dk is None else torch.tensor(wl.dk, dtype=torch.float64, requires_grad=True)
    out = autograd.ssfm(x, params, wl.nz, dk=dk, checkpoint_every=every, pass_order=order)
    loss = _loss([o.to(torch.complex128) for o in out])
    loss.backward()
    g = [t.grad.cpu().numpy() for t in x]
    gdk = None if dk is None else dk.grad.numpy()
    return float(loss), g, gdk, [o.detach().cpu().numpy() for o in out]


def _oracle_grads(wl):
    prob = oracle_problem(wl)
    dk = list(wl.dk) if wl.dk is not None else [wl.dk_const] * wl.nz
    prob.dk = dk
    loss = lambda out, p: -(out[-1].abs() ** 2).sum()
    j, g, gdk = oadj.gradients([torch.from_numpy(a) for a in wl.init], dk, prob, wl.nz, loss=loss)
    return j, [x.numpy() for x in g], gdk.numpy()


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("nf,shape,nz,every", [(2, (16, 16, 8), 12, 5), (3, (8, 16, 16), 9, 4),
                                                (2, (32, 8, 16), 7, 7), (3, (24, 12, 6), 8, 3),
                                                (3, (18, 9, 36), 8, 3), (2, (36, 18, 9), 7, 4),
                                                # 36 values per lane on x and tau, ragged tiles
                                                (3, (144, 4, 72), 6, 3),
                                                # reduced dimensions: the forward leaves out the
                                                # passes along length-1 axes, the reverse sweep not
                                                (2, (32, 16, 1), 10, 4), (3, (1, 1, 64), 11, 5)])
def test_adjoint_matches_oracle(nf, shape, nz, every, order):
    wl = _case(nf, shape, nz, seed=nf * 10 + nz)
    jg, g, gdk, _ = _gpu_grads(wl, every, order)
    jo, go, gdko = _oracle_grads(wl)
    assert abs(jg - jo) < 1e-5 * abs(jo)
    for j in range(nf):
        assert rel_l2(g[j], go[j]) < 1e-4, j
    assert rel_l2(gdk, gdko) < 1e-4


def test_adjoint_constant_dk_is_sum_of_profile_gradient():
    wl = _case(2, (16, 8, 8), 10, seed=3, profile=False)
    params = brahms.params_from_workload(wl)
    fields = [torch.from_numpy(a).to(DEV) for a in wl.init]
    plan = brahms.Plan(wl.nx, wl.ny, wl.nt, 2, params).bind(fields)
    plan.adjoint_forward(wl.nz, 4)
    g = [torch.zeros_like(f) for f in fields]
    g[1].copy_(-2 * fields[1])   # dJ/dS* convention of J = -sum |S|^2
    gdk = plan.adjoint_backward(g)
    _, _, gdko = _oracle_grads(wl)
    assert gdk.shape == (1,)
    assert abs(gdk[0] - gdko.sum()) < 1e-4 * abs(gdko.sum())


def test_adjoint_forward_equals_plain_step():
    wl = _case(3, (16, 16, 16), 11, seed=4)
    params = brahms.params_from_workload(wl)
    a = [torch.from_numpy(x).to(DEV) for x in wl.init]
    b = [x.clone() for x in a]
    p1 = brahms.Plan(16, 16, 16, 3, params).bind(a)
    p1.step(wl.nz)
    p2 = brahms.Plan(16, 16, 16, 3, params).bind(b)
    p2.adjoint_forward(wl.nz, 4)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert abs(p2.z - p1.z) < 1e-15


@pytest.mark.parametrize("order", [0, 1])
def test_inverse_design_workload_vs_oracle(order):
    """SHG 128x128x64, 400 steps, per-step dk = 2/L + N(0, 0.1/L), checkpoints
    every 20 steps, J = -sum |S(L)|^2: the loss, dJ/ddk (all 400 entries) and
    sampled dJ/dF_in against the oracle's adjoint (tests/golden)."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "shg_adjoint_grad.npz"))
    wl = inputs.shg_adjoint()
    params = brahms.params_from_workload(wl)
    x = [torch.from_numpy(a).to(DEV).requires_grad_(True) for a in wl.init]
    dk = torch.tensor(wl.dk, dtype=torch.float64, requires_grad=True)
    out = autograd.ssfm(x, params, wl.nz, dk=dk, checkpoint_every=20, pass_order=order)
    loss = -(out[1].to(torch.complex128).abs() ** 2).sum()
    loss.backward()
    assert abs(float(loss) - float(g["J"])) < 2e-5 * abs(float(g["J"]))
    assert rel_l2(dk.grad.numpy(), g["grad_dk"]) < 1e-4
    gf = x[0].grad.cpu().numpy().reshape(-1)
    assert rel_l2(gf[g["uniform_idx"]], g["gF_uniform"]) < 1e-4
    assert rel_l2(gf[g["top_idx"]], g["gF_top"]) < 1e-4
    # the whole gradient: relative L2 estimated from a count sketch of every
    # grid value (tests/sketch.py; seed 8000 as in make_adjoint_golden.py)
    ref = g["gF_sketch"].astype(np.complex128)
    est = float(np.linalg.norm(count_sketch(gf, ref.size, 8000) - ref) / np.sqrt(g["gF_norm2"]))
    assert est < 1e-4, est
    power = (np.abs(x[0].grad.cpu().numpy().astype(np.complex128)) ** 2).sum(axis=(1, 2))
    assert rel_l2(power, g["gF_power"]) < 2e-4


def test_inverse_design_forward_fields_vs_oracle():
    """The forward fields of the inverse-design workload (SHG 128 x 128 x 64,
    400 steps, per-step dk profile) at z = L: <= 2e-5 per field against the
    oracle's reference data, from the plain plan and from the checkpointed
    forward of the adjoint."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "shg_adjoint_400.npz")
    if not os.path.exists(path):
        pytest.skip("reference data not generated")
    g = np.load(path)
    wl = inputs.shg_adjoint()
    params = brahms.params_from_workload(wl)
    for adjoint in (False, True):
        fields = [torch.from_numpy(a).to(DEV) for a in wl.init]
        plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, params).bind(fields)
        if adjoint:
            plan.adjoint_forward(wl.nz, 20)
        else:
            plan.step(wl.nz)
        torch.cuda.synchronize()
        for j, f in enumerate(fields):
            flat = f.cpu().numpy().reshape(-1)
            # whole field, from the count sketch (seed 7000 + j, make_golden.py)
            ref = g[f"f{j}_sketch"].astype(np.complex128)
            est = float(np.linalg.norm(count_sketch(flat, ref.size, 7000 + j) - ref) / np.sqrt(g["energies"][j]))
            assert est < 2e-5, (adjoint, j, est)
            assert rel_l2(flat[g["uniform_idx"]], g[f"f{j}_uniform"]) < 2e-5, (adjoint, j)
            assert rel_l2(flat[g[f"f{j}_top_idx"]], g[f"f{j}_top"]) < 2e-5, (adjoint, j)
        plan.destroy()


@pytest.mark.parametrize("alias", [False, True])
def test_one_call_adjoint_equals_split_calls(alias):
    """brahms_adjoint (fields in, cotangent out -> cotangent in, dJ/ddk in
    one call) gives the bits of brahms_adjoint_forward + _backward, with
    separate or aliased buffers; the bound fields end at the forward output."""
    wl = _case(3, (16, 8, 16), 11, seed=5)
    params = brahms.params_from_workload(wl)
    rng = np.random.default_rng(9)
    gout = [torch.from_numpy((rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape))
                             .astype(np.complex64)).to(DEV) for a in wl.init]
    # split calls
    f1 = [torch.from_numpy(a).to(DEV) for a in wl.init]
    p1 = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, params).bind(f1)
    p1.adjoint_forward(wl.nz, 4)
    g1 = [g.clone() for g in gout]
    gdk1 = p1.adjoint_backward(g1)
    torch.cuda.synchronize()
    # one call
    bound = [torch.zeros_like(f) for f in f1]
    p2 = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, params).bind(bound)
    fin = [torch.from_numpy(a).to(DEV) for a in wl.init]
    if alias:
        for b, a in zip(bound, fin):
            b.copy_(a)
        fin = bound
        g2 = [g.clone() for g in gout]
        gdk2 = p2.adjoint(wl.nz, 4, fin, g2, g2)
    else:
        g2 = [torch.zeros_like(g) for g in gout]
        gdk2 = p2.adjoint(wl.nz, 4, fin, gout, g2)
    torch.cuda.synchronize()
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
    assert np.array_equal(gdk1, gdk2)
    for a, b in zip(f1, bound):
        assert torch.equal(a, b)
    p1.destroy()
    p2.destroy()
