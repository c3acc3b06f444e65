"""GPU parity: the HIP engine (through the C ABI) against the FP64 oracle on
the same seeded complex64 inputs.  Tolerances are relative L2 per field."""
import math
import os

import numpy as np
import pytest
import torch

from paper_2609_08384_amd import brahms, inputs
from tests.sketch import count_sketch
from tests.util import oracle_run, rel_l2

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
EPS32 = 2.0 ** -24


def _accumulation_bound(n_updates, scale):
    """Worst case of storing a complex64 state after each of n_updates
    increments: n_updates half-ulps (sqrt 2 for complex) of the largest
    magnitude reached.  Constant increments (plane waves) make these
    rounding errors coherent, so this, not sqrt(n), is the bound to test."""
    return n_updates * EPS32 * math.sqrt(2.0) * scale


def _wl(nx, ny, nt, nf, nz, dz, fields, dk_const=0.0, dk=None, init=None):
    wl = inputs.Workload("case", nx, ny, nt, nf, nz, dz, fields, dk_const=dk_const, dk=dk)
    wl.init = init
    return wl


def _gpu(wl, nsteps=None, pass_order=None, merge=0, fuse=0):
    out = brahms.run_workload(wl, nsteps=nsteps, device=DEV, pass_order=pass_order, merge_halves=merge,
                              fuse_steps=fuse)
    return [f.cpu().numpy() for f in out]


def _oracle(wl, nsteps=None, merge=0):
    return [a.numpy() for a in oracle_run(wl, nsteps, merge=bool(merge))]


def _all_terms(nf, scale=1.0, kappa=0.0):
    base = [dict(diffraction=1.7, tan_rho=0.9, delay=-1.3, k2=2.1, k3=0.7, alpha=0.2),
            dict(diffraction=0.8, tan_rho=-0.4, delay=0.6, k2=-1.5, k3=-0.3, alpha=0.0),
            dict(diffraction=2.6, tan_rho=0.2, delay=1.1, k2=0.9, k3=0.2, alpha=0.1)]
    return [inputs.FieldSpec(kappa=kappa * (1 - 0.2 * j), **{k: v * scale for k, v in base[j].items()})
            for j in range(nf)]


SHAPES = [(32, 16, 8), (16, 32, 64), (64, 8, 4), (96, 64, 2), (128, 4, 16), (256, 2, 1),
          (1, 1, 256), (8, 256, 1), (4, 96, 32), (2, 128, 8), (1, 4, 128), (128, 96, 96),
          # the lengths 3 * 2^a
          (3, 6, 12), (24, 48, 3), (192, 4, 6), (6, 192, 2), (12, 24, 192), (48, 3, 24),
          # the lengths 9 * 2^a
          (9, 18, 36), (72, 144, 2), (144, 9, 18), (36, 72, 9), (18, 4, 144), (2, 144, 72),
          (144, 144, 144)]


@pytest.mark.parametrize("shape", SHAPES)
def test_linear_step_each_axis_length(shape):
    """kappa = 0: one step is the linear step alone (FFT, propagator, inverse)."""
    nx, ny, nt = shape
    rng = np.random.default_rng(sum(shape))
    init = inputs.random_fields(rng, 3, nx, ny, nt)
    wl = _wl(nx, ny, nt, 3, 1, 0.05, _all_terms(3), init=init)
    g, o = _gpu(wl), _oracle(wl)
    for j in range(3):
        assert rel_l2(g[j], o[j]) < 2e-6, (shape, j)


@pytest.mark.parametrize("merge", [0, 1])
def test_plane_wave_depleted_shg(merge):
    """Uniform fields: only the k = 0 mode, so the loop is the RK4 half-steps
    alone; depleted SHG has F = F0 sech(G z), S = i sqrt(kS/kF) F0 tanh(G z)
    (also with adjacent halves merged into RK4 steps of size dz)."""
    kf, ks, f0, nz = 1.3, 0.6, 1.5, 100
    init = [np.full((4, 4, 4), f0, np.complex64), np.zeros((4, 4, 4), np.complex64)]
    wl = _wl(4, 4, 4, 2, nz, 1.0 / nz, [inputs.FieldSpec(kappa=kf), inputs.FieldSpec(kappa=ks)], init=init)
    f, s = _gpu(wl, merge=merge)
    g = math.sqrt(kf * ks) * f0
    bound = _accumulation_bound(2 * nz, f0)
    assert np.abs(f - f0 / math.cosh(g)).max() < bound
    assert np.abs(s - 1j * math.sqrt(ks / kf) * f0 * math.tanh(g)).max() < bound


@pytest.mark.parametrize("dk", [0.0, 3.0, -7.5])
def test_plane_wave_undepleted_shg_sinc(dk):
    f0, ks, nz = 0.8 + 0.3j, 1.7, 100
    init = [np.full((2, 2, 2), f0, np.complex64), np.zeros((2, 2, 2), np.complex64)]
    wl = _wl(2, 2, 2, 2, nz, 1.0 / nz, [inputs.FieldSpec(kappa=0.0), inputs.FieldSpec(kappa=ks)],
             dk_const=dk, init=init)
    f, s = _gpu(wl)
    integral = 1.0 if dk == 0 else (1 - np.exp(-1j * dk)) / (1j * dk)
    want = 1j * ks * complex(np.complex64(f0)) ** 2 * integral
    bound = _accumulation_bound(2 * nz, ks * abs(f0) ** 2) + 1e-7
    assert np.abs(s - want).max() < bound


def test_plane_wave_opa():
    ap, as0, ks, ki, nz = 1.2 * np.exp(0.4j), 0.01 - 0.02j, 1.5, 0.9, 100
    init = [np.full((2, 4, 2), ap, np.complex64), np.full((2, 4, 2), as0, np.complex64),
            np.zeros((2, 4, 2), np.complex64)]
    wl = _wl(2, 4, 2, 3, nz, 1.0 / nz, [inputs.FieldSpec(kappa=0.0), inputs.FieldSpec(kappa=ks),
                                         inputs.FieldSpec(kappa=ki)], init=init)
    p, s, i = _gpu(wl)
    ap, as0 = complex(np.complex64(ap)), complex(np.complex64(as0))
    g = math.sqrt(ks * ki) * abs(ap)
    ws = as0 * math.cosh(g)
    wi = 1j * ki * ap * np.conj(as0) * math.sinh(g) / g
    assert np.abs(s - ws).max() < _accumulation_bound(2 * nz, abs(ws)) + 1e-7 * abs(ws)
    assert np.abs(i - wi).max() < _accumulation_bound(2 * nz, abs(wi)) + 1e-7 * abs(wi)


@pytest.mark.parametrize("merge", [0, 1])
@pytest.mark.parametrize("order", [0, 1, 2, 3])
@pytest.mark.parametrize("nf,shape", [(2, (32, 32, 32)), (3, (32, 32, 32)), (3, (64, 16, 96)),
                                      (2, (96, 96, 4)), (3, (16, 128, 64)), (3, (48, 24, 12)),
                                      (2, (192, 6, 24)), (3, (12, 192, 3)), (3, (36, 18, 72)),
                                      (2, (144, 9, 16)), (3, (18, 144, 9))])
def test_coupled_steps_random(nf, shape, order, merge):
    """All linear terms and the chi(2) coupling, 10 steps, ragged tiles, every
    pass order, literal and merged half-steps."""
    nx, ny, nt = shape
    rng = np.random.default_rng(100 + nf)
    init = inputs.random_fields(rng, nf, nx, ny, nt, scale=0.7, smooth=min(nx, ny, nt) / 2.0)
    wl = _wl(nx, ny, nt, nf, 10, 0.02, _all_terms(nf, kappa=1.5), dk_const=2.3, init=init)
    g, o = _gpu(wl, pass_order=order, merge=merge), _oracle(wl, merge=merge)
    for j in range(nf):
        assert rel_l2(g[j], o[j]) < 5e-6, j


@pytest.mark.parametrize("fuse", [0, 1])
@pytest.mark.parametrize("shape", [(8, 12, 16), (24, 32, 48), (64, 16, 24), (48, 64, 8), (12, 8, 64)])
def test_second_splits_match_oracle(shape, fuse):
    """The second register/lane split of every length that has one
    (schedule field split, all three axes), three fields, literal and fused
    schedules, against the oracle; and it really is another kernel (the bits
    differ from the first split's)."""
    nx, ny, nt = shape
    rng = np.random.default_rng(500 + sum(shape))
    init = inputs.random_fields(rng, 3, nx, ny, nt, scale=0.7, smooth=min(nx, ny, nt) / 2.0)
    wl = _wl(nx, ny, nt, 3, 9, 0.02, _all_terms(3, kappa=1.5), dk_const=2.3, init=init)
    merge = fuse
    out = brahms.run_workload(wl, device=DEV, pass_order=0, merge_halves=merge, fuse_steps=fuse, split=7)
    g = [f.cpu().numpy() for f in out]
    o = _oracle(wl, merge=merge)
    for j in range(3):
        assert rel_l2(g[j], o[j]) < 5e-6, j
    first = _gpu(wl, pass_order=0, merge=merge, fuse=fuse)
    assert any(not np.array_equal(a, b) for a, b in zip(g, first))


@pytest.mark.parametrize("shape", [(32, 16, 8), (1, 1, 256), (256, 2, 1), (8, 96, 1), (96, 64, 2)])
def test_merged_half_steps_differ_from_literal_by_truncation_only(shape):
    """Merged halves really run (the bits differ from the literal splitting)
    and match the oracle's merged loop; every pass structure (three passes,
    the single tau pass of nx = ny = 1, CW grids)."""
    nx, ny, nt = shape
    rng = np.random.default_rng(sum(shape))
    init = inputs.random_fields(rng, 3, nx, ny, nt, scale=0.7, smooth=max(1.0, min(nx, ny, nt) / 2.0))
    wl = _wl(nx, ny, nt, 3, 40, 0.02, _all_terms(3, kappa=1.5), dk_const=-1.7, init=init)
    lit, mer, o = _gpu(wl), _gpu(wl, merge=1), _oracle(wl, merge=1)
    assert any(not np.array_equal(a, b) for a, b in zip(lit, mer))
    for j in range(3):
        assert rel_l2(mer[j], o[j]) < 5e-6, j


def test_dk_profile_matches_oracle():
    rng = np.random.default_rng(9)
    nx = ny = nt = 16
    init = inputs.random_fields(rng, 2, nx, ny, nt, scale=0.8, smooth=6.0)
    dk = 2.0 + rng.standard_normal(40)
    wl = _wl(nx, ny, nt, 2, 40, 0.025, _all_terms(2, kappa=1.0), dk=dk, init=init)
    g, o = _gpu(wl), _oracle(wl)
    for j in range(2):
        assert rel_l2(g[j], o[j]) < 5e-6


@pytest.mark.parametrize("merge,fuse", [(0, 0), (1, 0), (1, 1)])
@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_shg32_full_run(order, merge, fuse):
    """SHG 32^3, 100 steps (the small benchmark workload): <= 1e-5 per field."""
    wl = inputs.shg32()
    g, o = _gpu(wl, pass_order=order, merge=merge, fuse=fuse), _oracle(wl, merge=merge)
    for j in range(2):
        assert rel_l2(g[j], o[j]) < 1e-5, j


def test_deterministic_and_resumable():
    """Two identical runs agree bitwise (no races, no atomics in the step),
    and 30 + 20 steps through set_z equal 50 steps in one call."""
    wl = inputs.shg32()
    a = _gpu(wl, 50)
    b = _gpu(wl, 50)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    fields = [torch.from_numpy(x).to(DEV) for x in wl.init]
    plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, brahms.params_from_workload(wl)).bind(fields)
    plan.propagate(30 * wl.dz)
    saved = [f.clone() for f in fields]
    plan.destroy()
    plan2 = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, brahms.params_from_workload(wl)).bind(saved)
    plan2.set_z(30 * wl.dz)
    assert abs(plan2.z - 0.3) < 1e-12
    plan2.propagate(0.5)
    torch.cuda.synchronize()
    for x, y in zip(saved, a):
        assert np.array_equal(x.cpu().numpy().view(np.uint8), y.view(np.uint8))


def test_plan_on_a_side_stream():
    """A plan created on a non-current stream (its workspace allocated for
    that stream) gives the bits of a plan on the current stream."""
    wl = inputs.shg32()
    ref = _gpu(wl, 30)
    side = torch.cuda.Stream()
    fields = [torch.from_numpy(a).to(DEV) for a in wl.init]
    torch.cuda.synchronize()
    plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, brahms.params_from_workload(wl), stream=side)
    plan.bind(fields)
    plan.step(30)
    side.synchronize()
    for a, b in zip(fields, ref):
        assert np.array_equal(a.cpu().numpy().view(np.uint8), b.view(np.uint8))
    plan.destroy()


@pytest.mark.parametrize("nf,shape", [(3, (32, 16, 8)), (2, (96, 64, 2)), (3, (24, 48, 192)), (2, (256, 2, 1)),
                                      (3, (16, 128, 64)), (2, (3, 6, 12)), (3, (128, 96, 96)),
                                      # 72 and 144 have no wide form: their bits are ignored
                                      (3, (144, 72, 36)), (2, (18, 9, 144))])
@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_wide_linear_passes_bitwise(nf, shape, order):
    """512-thread blocks for the linear passes (schedule field `wide`, every
    axis) transform every line as the 256-thread blocks do: the same bits,
    literal, merged and fused, over calls that cross a 64-step chunk, with
    partial last blocks (lines not a multiple of the lines per block)."""
    nx, ny, nt = shape
    rng = np.random.default_rng(700 + nf + nt + order)
    init = inputs.random_fields(rng, nf, nx, ny, nt, scale=0.6, smooth=max(1.0, min(shape) / 2.0))
    wl = _wl(nx, ny, nt, nf, 70, 0.01, _all_terms(nf, kappa=1.4), dk_const=1.7, init=init)
    for merge, fuse in ((0, 0), (1, 0), (1, 1)):
        ref = brahms.run_workload(wl, device=DEV, pass_order=order, merge_halves=merge, fuse_steps=fuse)
        out = brahms.run_workload(wl, device=DEV, pass_order=order, merge_halves=merge, fuse_steps=fuse,
                                  wide=7)
        for a, b in zip(out, ref):
            assert torch.equal(a, b), (merge, fuse)


def test_opg256_wide_middle_pass_bitwise():
    """The benchmark workload with its middle (y) pass on 512-thread blocks:
    the bits of 256-thread blocks after 12 fused steps."""
    wl = inputs.opg256()
    ref = brahms.run_workload(wl, 12, device=DEV, pass_order=0, merge_halves=1, fuse_steps=1)
    out = brahms.run_workload(wl, 12, device=DEV, pass_order=0, merge_halves=1, fuse_steps=1, wide=2)
    for a, b in zip(out, ref):
        assert torch.equal(a, b)


def test_nonfinite_detected():
    """A dz far too large for kappa |A| (Sec. 3.2) blows the fields up; with
    BRAHMS_CHECK_FINITE the call reports E_NONFINITE."""
    init = [np.full((8, 8, 8), 30.0, np.complex64), np.full((8, 8, 8), 30.0, np.complex64)]
    p = brahms.Params(dz=0.5, fields=[brahms.FieldParams(kappa=50.0), brahms.FieldParams(kappa=50.0)],
                      check_finite=True)
    fields = [torch.from_numpy(a).to(DEV) for a in init]
    plan = brahms.Plan(8, 8, 8, 2, p).bind(fields)
    with pytest.raises(brahms.BrahmsError) as ei:
        plan.step(40)
    assert ei.value.status == brahms.BRAHMS_E_NONFINITE
    plan.destroy()


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check_golden(out, name, tol, prefix=""):
    """Compare a GPU run with the oracle reference data written by
    tests/golden/make_golden.py: the whole-field relative L2 error per field,
    estimated from a count sketch of every grid value (tests/sketch.py), and
    the sampled values, power traces P(tau), fluence maps and energies.  The
    data are those of the literal loop; at the step sizes of these workloads
    the merged loop differs from it by ~1e-11 (FP64), so they serve merged
    runs too.  Returns the reference data and the whole-field estimates."""
    g = np.load(f"{GOLDEN}/{name}.npz")
    whole = []
    for j, a in enumerate(out):
        if f"{prefix}f{j}_sketch" in g.files:
            ref = g[f"{prefix}f{j}_sketch"].astype(np.complex128)
            est = float(np.linalg.norm(count_sketch(a, ref.size, SKETCH_SEED + j) - ref) /
                        np.sqrt(g[f"{prefix}energies"][j]))
            whole.append(est)
            assert est < tol, (j, "whole field (sketch)", est)
        if prefix:
            continue
        flat = a.reshape(-1)
        assert rel_l2(flat[g["uniform_idx"]], g[f"f{j}_uniform"]) < tol, (j, "uniform")
        assert rel_l2(flat[g[f"f{j}_top_idx"]], g[f"f{j}_top"]) < tol, (j, "top")
        inten = np.abs(a.astype(np.complex128)) ** 2
        assert rel_l2(inten.sum(axis=(1, 2)), g[f"f{j}_power"]) < 2 * tol, (j, "power")
        nt, ny, nx = a.shape
        by, bx = max(1, ny // 64), max(1, nx // 64)
        flu = inten.sum(axis=0).reshape(ny // by, by, nx // bx, bx).sum(axis=(1, 3))
        assert rel_l2(flu, g[f"f{j}_fluence"]) < 2 * tol, (j, "fluence")
    return g, whole


SKETCH_SEED = 7000   # the seed tests/golden/make_golden.py sketches field j with (+ j)


# (pass order, merged half-steps, fused step pairs)
SCHEDULES = [(o, m, f) for m, f in ((0, 0), (1, 0), (1, 1)) for o in range(4)]


@pytest.mark.parametrize("order,merge,fuse", SCHEDULES)
def test_sfg128_full_run_vs_oracle(order, merge, fuse):
    """SFG 128^3, 500 steps, pump depletion: <= 2e-5 per field."""
    wl = inputs.sfg128()
    out = _gpu(wl, pass_order=order, merge=merge, fuse=fuse)
    g, whole = _check_golden(out, "sfg128_500", 2e-5)
    assert len(whole) == 3
    e = [float((np.abs(a.astype(np.complex128)) ** 2).sum()) for a in out]
    assert np.allclose(e, g["energies"], rtol=4e-5)


@pytest.mark.parametrize("order,merge,fuse", SCHEDULES)
def test_opg256_first_steps_vs_oracle(order, merge, fuse):
    """OPG 256^3 (the benchmark workload), first 10 steps at full size, in the
    launch configurations the benchmark may time: <= 3e-5 per field."""
    wl = inputs.opg256()
    out = _gpu(wl, 10, pass_order=order, merge=merge, fuse=fuse)
    _check_golden(out, "opg256_10", 3e-5)


@pytest.mark.parametrize("order,merge,fuse", SCHEDULES)
def test_opg256_full_run_vs_oracle(order, merge, fuse):
    """OPG 256^3, all 1000 steps (the benchmark workload end to end, in both
    launch configurations the benchmark may time): <= 3e-5 per field on the
    sampled values, power traces and fluence maps; energies and Manley-Rowe
    combinations of the oracle."""
    if not os.path.exists(f"{GOLDEN}/opg256_1000.npz"):
        pytest.skip("reference data not generated")
    wl = inputs.opg256()
    out = _gpu(wl, pass_order=order, merge=merge, fuse=fuse)
    g, whole = _check_golden(out, "opg256_1000", 3e-5)
    assert len(whole) == 3
    e = [float((np.abs(a.astype(np.complex128)) ** 2).sum()) for a in out]
    assert np.allclose(e, g["energies"], rtol=6e-5)


@pytest.mark.parametrize("order", [0, 1])
def test_opg256_full_run_in_the_benchmark_schedule(order):
    """OPG 256^3, all 1000 steps, in the schedule the benchmark's tuner picks
    (merged half-steps, fused step pairs, the middle y pass on 512-thread
    blocks): the same bounds as the other full runs, over the whole fields."""
    if not os.path.exists(f"{GOLDEN}/opg256_1000.npz"):
        pytest.skip("reference data not generated")
    wl = inputs.opg256()
    out = [f.cpu().numpy() for f in brahms.run_workload(wl, device=DEV, pass_order=order, merge_halves=1,
                                                          fuse_steps=1, wide=2)]
    g, whole = _check_golden(out, "opg256_1000", 3e-5)
    assert len(whole) == 3


def test_error_grows_like_sqrt_of_steps():
    """Rounding along z (reading T of the design notes): with the propagator
    phases telescoped and every per-step constant rounded afresh, the GPU's
    errors are independent from step to step and add up like a random walk,
    so the error at 10 %, 50 % and 100 % of the 500 steps of the SFG 128^3
    workload grows like sqrt(steps) (exponent 1/2), not like the steps
    (exponent 1, a coherent per-step error).  Measured on the whole fields
    (count sketches of the oracle's fields at steps 50, 250 and 500), as the
    total error over the three fields relative to their total norm."""
    g = np.load(f"{GOLDEN}/sfg128_500.npz")
    wl = inputs.sfg128()
    fields = [torch.from_numpy(a).to(DEV) for a in wl.init]
    plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, brahms.params_from_workload(wl))
    plan.set_schedule(0, 0, 1, 1)
    plan.bind(fields)
    total = {}
    for n in (50, 250, 500):
        plan.propagate(n * wl.dz)
        torch.cuda.synchronize()
        prefix = "" if n == 500 else f"s{n}_"
        err2 = norm2 = 0.0
        for j, f in enumerate(fields):
            ref = g[f"{prefix}f{j}_sketch"].astype(np.complex128)
            err2 += float(np.linalg.norm(count_sketch(f.cpu().numpy(), ref.size, SKETCH_SEED + j) - ref)) ** 2
            norm2 += float(g[f"{prefix}energies"][j])
        total[n] = math.sqrt(err2 / norm2)
        assert total[n] < 2e-5, (n, total[n])
    plan.destroy()
    p10 = math.log(total[500] / total[50]) / math.log(10.0)
    p5 = math.log(total[250] / total[50]) / math.log(5.0)
    print(f"total relative error at 50/250/500 steps: {total}; growth exponents {p5:.2f}, {p10:.2f}")
    # midway (on a log scale) between sqrt growth and linear growth
    assert p10 < 0.75 and p5 < 0.75, (total, p5, p10)


def test_opg256_first_steps_whole_field_vs_oracle():
    """OPG 256^3 (the benchmark workload), 10 steps in the benchmark's launch
    configuration (merged half-steps, fused step pairs), every grid value of
    every field against the oracle's merged loop run here on the host: the
    relative L2 error of each whole field within the 3e-5 tolerance, and no
    single value off by more than 3e-5 of the field's largest amplitude."""
    wl = inputs.opg256()
    out = _gpu(wl, 10, pass_order=0, merge=1, fuse=1)
    ref = _oracle(wl, 10, merge=1)
    for j, (a, r) in enumerate(zip(out, ref)):
        assert rel_l2(a, r) < 3e-5, j
        assert np.max(np.abs(a.astype(np.complex128) - r)) < 3e-5 * np.max(np.abs(r)), j


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_graph_schedule_is_bitwise_eager(order):
    """Whole 64-step chunks replayed from the plan's hipGraph give the same
    bits as launch-by-launch stepping: ragged call lengths, a per-step dk
    profile and a transverse map (chunk tables), a resume with set_z, a
    monitor switched on in between (those chunks run eagerly) and a rebind to
    new tensors (the graph is captured again)."""
    rng = np.random.default_rng(77)
    nz = 500
    fs = [inputs.FieldSpec(kappa=1.2, diffraction=0.8, tan_rho=0.3, k2=0.5),
          inputs.FieldSpec(kappa=0.9, diffraction=0.4, delay=-0.6, k2=-0.7),
          inputs.FieldSpec(kappa=0.5, diffraction=1.1, delay=0.4, k2=0.2)]
    wl = inputs.Workload("g", 32, 16, 8, 3, nz, 1.0 / nz, fs, dk=2.0 + rng.standard_normal(nz),
                         dk_map=rng.uniform(-5, 5, (16, 32)))
    wl.init = inputs.random_fields(rng, 3, 32, 16, 8, scale=0.5, smooth=6.0)
    params = brahms.params_from_workload(wl)

    def run(graph, calls):
        f = [torch.from_numpy(a).to(DEV) for a in wl.init]
        plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, params)
        plan.set_schedule(order, graph)
        plan.bind(f)
        for c in calls:
            if c == "monitor":
                plan.set_monitor(10, capacity=8)
            elif c == "nomonitor":
                plan.set_monitor(0)
            elif c == "rebind":
                f = [x.clone() for x in f]
                plan.bind(f)
            elif isinstance(c, tuple):
                plan.set_z(c[1] * wl.dz)
            else:
                plan.step(c)
        torch.cuda.synchronize()
        out = [x.clone() for x in f]
        plan.destroy()
        return out

    calls = [70, 64, ("z", 100), 128, "monitor", 64, "nomonitor", "rebind", 64, 5, 69]
    eager = run(0, calls)
    graph = run(1, calls)
    for a, b in zip(eager, graph):
        assert torch.equal(a, b)


@pytest.mark.parametrize("fuse", [0, 1])
@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_graph_schedule_with_merged_halves_is_bitwise_eager(order, fuse):
    """Merged half-steps: graph replays (which continue a call, so a call's
    first chunk runs eagerly) give the bits of launch-by-launch stepping over
    ragged calls, a resume, a monitor (whose calls keep literal half-steps)
    and a rebind; and merged calls differ from literal ones."""
    rng = np.random.default_rng(78)
    nz = 500
    fs = [inputs.FieldSpec(kappa=1.2, diffraction=0.8, tan_rho=0.3, k2=0.5),
          inputs.FieldSpec(kappa=0.9, diffraction=0.4, delay=-0.6, k2=-0.7),
          inputs.FieldSpec(kappa=0.5, diffraction=1.1, delay=0.4, k2=0.2)]
    wl = inputs.Workload("g", 32, 16, 8, 3, nz, 1.0 / nz, fs, dk_const=2.5)
    wl.init = inputs.random_fields(rng, 3, 32, 16, 8, scale=0.5, smooth=6.0)
    params = brahms.params_from_workload(wl)

    def run(graph, merge, calls):
        f = [torch.from_numpy(a).to(DEV) for a in wl.init]
        plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, params)
        plan.set_schedule(order, graph, merge, fuse if merge else 0)
        plan.bind(f)
        for c in calls:
            if c == "monitor":
                plan.set_monitor(10, capacity=8)
            elif c == "nomonitor":
                plan.set_monitor(0)
            elif c == "rebind":
                f = [x.clone() for x in f]
                plan.bind(f)
            elif isinstance(c, tuple):
                plan.set_z(c[1] * wl.dz)
            else:
                plan.step(c)
        torch.cuda.synchronize()
        out = [x.clone() for x in f]
        plan.destroy()
        return out

    calls = [200, 64, ("z", 100), 129, "monitor", 64, "nomonitor", "rebind", 64, 5, 140]
    eager = run(0, 1, calls)
    graph = run(1, 1, calls)
    for a, b in zip(eager, graph):
        assert torch.equal(a, b)
    literal = run(0, 0, calls)
    for a, b in zip(eager, literal):
        assert not torch.equal(a, b)
        # ~730 steps: the two differ by their FP32 rounding (each ~1e-5 of
        # the exact result at this length), the truncation term is ~1e-11
        assert float((a - b).norm() / b.norm()) < 2e-5
    # with a monitor set the calls keep literal half-steps: the same bits as
    # a plan without merging
    mon = ["monitor", 70]
    for a, b in zip(run(0, 1, mon), run(0, 0, mon)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("order", [0, 1, 2, 3])
@pytest.mark.parametrize("nf,shape", [(3, (32, 32, 32)), (3, (64, 16, 96)), (2, (96, 96, 4)),
                                      (3, (16, 128, 64)), (2, (256, 2, 1)), (3, (8, 96, 1)),
                                      (3, (24, 48, 192)), (3, (72, 36, 18)), (2, (18, 144, 36))])
def test_fused_step_pairs_match_merged_oracle(nf, shape, order):
    """Fused step pairs (alternating axis orders, step n's last transform,
    the RK4 step and step n+1's first transform in one pass) compute the
    merged loop: against the oracle's merged loop, for call lengths that
    end on an even or odd step and that cross a 64-step table chunk."""
    nx, ny, nt = shape
    rng = np.random.default_rng(300 + nf + nt)
    init = inputs.random_fields(rng, nf, nx, ny, nt, scale=0.7, smooth=max(1.0, min(nx, ny, nt) / 2.0))
    for nz in (1, 2, 7, 66):
        wl = _wl(nx, ny, nt, nf, nz, 0.01, _all_terms(nf, kappa=1.5), dk_const=2.3, init=init)
        g, o = _gpu(wl, pass_order=order, merge=1, fuse=1), _oracle(wl, merge=1)
        for j in range(nf):
            assert rel_l2(g[j], o[j]) < 5e-6, (nz, j)


@pytest.mark.parametrize("nf,shape", [(3, (32, 32, 32)), (2, (96, 64, 2)), (3, (24, 48, 12)), (2, (64, 16, 128)),
                                      (3, (256, 8, 4)), (3, (36, 72, 18)), (2, (144, 18, 9))])
def test_tuned_plans_match_oracle(nf, shape, tmp_path, monkeypatch):
    """Whatever schedule the autotuner picks for a shape (pass order, graph,
    merged halves, fused pairs, register/lane splits, wide linear passes),
    the plan computes the oracle's loop (the merged one when the schedule
    merges) to the fused-pair tolerance, over a call that crosses a 64-step
    table chunk."""
    from paper_2609_08384_amd import autotune
    monkeypatch.setenv("BRAHMS_CACHE_DIR", str(tmp_path))
    autotune._memo.clear()
    nx, ny, nt = shape
    rng = np.random.default_rng(900 + nf + nt)
    init = inputs.random_fields(rng, nf, nx, ny, nt, scale=0.7, smooth=max(1.0, min(nx, ny, nt) / 2.0))
    wl = _wl(nx, ny, nt, nf, 70, 0.01, _all_terms(nf, kappa=1.5), dk_const=2.3, init=init)
    fields = [torch.from_numpy(a).to(DEV) for a in wl.init]
    plan = brahms.Plan(nx, ny, nt, nf, brahms.params_from_workload(wl))
    sched = autotune.apply(plan, DEV)
    plan.bind(fields)
    plan.step(wl.nz)
    torch.cuda.synchronize()
    plan.destroy()
    autotune._memo.clear()
    ref = _oracle(wl, merge=sched.get("merge_halves", 0))
    for j in range(nf):
        assert rel_l2(fields[j].cpu().numpy(), ref[j]) < 5e-6, (sched, j)


def test_fused_step_pairs_refused_where_a_step_is_not_three_passes():
    wl = inputs.Workload("pw", 1, 1, 64, 2, 4, 0.1, _all_terms(2, kappa=1.0))
    plan = brahms.Plan(1, 1, 64, 2, brahms.params_from_workload(wl))
    with pytest.raises(brahms.BrahmsError) as ei:
        plan.set_schedule(0, 0, 1, 1)
    assert ei.value.status == brahms.BRAHMS_E_UNSUPPORTED
    plan.set_schedule(0, 0, 1, 0)
    plan.destroy()


def test_snapshots_suspend_merged_and_fused_schedules():
    """Snapshots look at the fields after single steps, so calls made while
    they are set run literal half-steps and three passes: the same bits as a
    plan with the literal schedule, and the snapshots match it too."""
    rng = np.random.default_rng(44)
    init = inputs.random_fields(rng, 3, 32, 16, 8, scale=0.6, smooth=4.0)
    wl = _wl(32, 16, 8, 3, 40, 0.02, _all_terms(3, kappa=1.5), dk_const=1.1, init=init)
    params = brahms.params_from_workload(wl)

    def run(merge, fuse):
        f = [torch.from_numpy(a).to(DEV) for a in init]
        plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, params)
        plan.set_schedule(0, 0, merge, fuse)
        assert plan.get_schedule()["fuse_steps"] == fuse
        plan.bind(f)
        snaps = plan.set_snapshots([5, 17])
        plan.step(30)
        torch.cuda.synchronize()
        out = [x.clone() for x in f] + [t.clone() for snap in snaps for t in snap]
        plan.destroy()
        return out

    for a, b in zip(run(1, 1), run(0, 0)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("merge,fuse", [(0, 0), (1, 0), (1, 1)])
def test_degenerate_calls_and_fields(merge, fuse):
    """Zero steps leave the fields and z untouched; all-zero fields stay
    exactly zero (every transform, propagator and RK4 product of zeros is
    zero); both under every schedule."""
    rng = np.random.default_rng(12)
    init = inputs.random_fields(rng, 3, 16, 32, 8, scale=0.6, smooth=4.0)
    wl = _wl(16, 32, 8, 3, 10, 0.02, _all_terms(3, kappa=1.5), dk_const=0.7, init=init)
    f = [torch.from_numpy(a).to(DEV) for a in init]
    plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, brahms.params_from_workload(wl))
    plan.set_schedule(1, 0, merge, fuse)
    plan.bind(f)
    plan.step(0)
    torch.cuda.synchronize()
    assert plan.z == 0.0
    for a, b in zip(f, init):
        assert np.array_equal(a.cpu().numpy(), b)
    for x in f:
        x.zero_()
    plan.step(7)
    torch.cuda.synchronize()
    assert abs(plan.z - 7 * wl.dz) < 1e-12
    for x in f:
        assert not torch.any(x != 0)
    plan.destroy()


def test_batch_member_with_no_steps_is_untouched():
    """A batch member with a step count of 0 keeps its fields, with merged
    half-steps and fused step pairs in the launches around it."""
    rng = np.random.default_rng(13)
    wls = []
    for nz in (0, 9, 4):
        init = inputs.random_fields(rng, 2, 16, 16, 16, scale=0.6, smooth=4.0)
        wls.append(_wl(16, 16, 16, 2, nz, 0.05, _all_terms(2, kappa=1.0), dk_const=0.4, init=init))
    batch = brahms.Batch([(w.nx, w.ny, w.nt, w.nf, brahms.params_from_workload(w), w.nz) for w in wls])
    batch.set_merge_halves(1)
    batch.set_fuse_steps(1)
    fields = [[torch.from_numpy(a).to(DEV) for a in w.init] for w in wls]
    batch.bind(fields)
    batch.run()
    torch.cuda.synchronize()
    batch.destroy()
    for a, b in zip(fields[0], wls[0].init):
        assert np.array_equal(a.cpu().numpy(), b)
    for w, fs in zip(wls[1:], fields[1:]):
        alone = brahms.run_workload(w, device=DEV, pass_order=0, merge_halves=1, fuse_steps=1)
        for a, b in zip(fs, alone):
            assert torch.equal(a, b)
