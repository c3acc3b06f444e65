"""Host-side logic that needs no GPU: the schedule autotuner's choice and
cache, and the benchmark's command-line contract."""
import json
import os
import subprocess
import sys

import pytest

from paper_2609_08384_amd import autotune, brahms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def fake_tuner(monkeypatch, tmp_path):
    monkeypatch.setenv("BRAHMS_CACHE_DIR", str(tmp_path))
    monkeypatch.setattr(autotune, "_arch", lambda device: "gfx950")
    autotune._memo.clear()
    calls = []

    def install(times):
        def measure(nx, ny, nt, nf, params, schedule, device="cuda:0", steps=64, warmup=3):
            calls.append(dict(schedule))
            return times.get((schedule["pass_order"], schedule["graph"], schedule["fuse_steps"]),
                             times.get((schedule["pass_order"], schedule["graph"]), 10.0))
        monkeypatch.setattr(autotune, "measure", measure)
        return calls
    yield install
    autotune._memo.clear()


def _params():
    return brahms.Params(dz=0.01, fields=[brahms.FieldParams(kappa=1.0)] * 2)


def test_tuner_takes_the_fastest_order_and_caches(fake_tuner, tmp_path):
    calls = fake_tuner({(0, 0): 1.0, (1, 0): 0.9, (0, 1): 0.95, (1, 1): 0.89})
    best = autotune.tune(32, 32, 32, 2, _params())
    # the graph is not 2 % faster than the best launch-by-launch order
    assert best == {"pass_order": 1, "graph": 0, "merge_halves": 1, "fuse_steps": 0}
    # constant dk: merged half-steps, with and without fused step pairs; a
    # warm-up run, then every candidate in each timing round, then the
    # register/lane splits of the three axes (length 32 has a second one)
    n_split = len(autotune.split_masks(32, 32, 32)) - 1
    assert n_split == 7
    # then 512-thread blocks on the linear axes (merged, unfused order 1:
    # tau first and y in the middle, alone and together)
    n_wide = len(autotune.wide_masks(best, 32, 32, 32))
    assert autotune.wide_masks(best, 32, 32, 32) == [2, 4, 6]
    # lengths 72 and 144 have no wide form: no bit on their axes
    assert autotune.wide_masks(best, 32, 72, 32) == [4]
    assert autotune.wide_masks(best, 32, 72, 144) == []
    n_calls = 1 + autotune.ROUNDS * (2 * len(autotune.CANDIDATES) + n_split + n_wide)
    assert len(calls) == n_calls
    assert all(c["merge_halves"] == 1 for c in calls)
    assert {c["fuse_steps"] for c in calls} == {0, 1}
    with open(os.path.join(str(tmp_path), "schedules.json")) as fh:
        disk = json.load(fh)
    (key, entry), = disk.items()
    assert key == "v8:gfx950:32x32x32:nf2:m1" and entry["schedule"] == best
    autotune._memo.clear()
    assert autotune.tune(32, 32, 32, 2, _params()) == best     # from the disk cache
    assert len(calls) == n_calls


def test_tuner_takes_the_graph_when_clearly_faster(fake_tuner):
    fake_tuner({(0, 0): 1.0, (1, 0): 1.1, (0, 1): 0.5, (1, 1): 0.6})
    assert autotune.tune(16, 16, 16, 3, _params(), refresh=True) == {
        "pass_order": 0, "graph": 1, "merge_halves": 1, "fuse_steps": 0}


def test_tuner_takes_fused_step_pairs_when_faster(fake_tuner):
    calls = fake_tuner({(0, 0, 0): 1.0, (2, 0, 1): 0.9})
    assert autotune.tune(32, 32, 32, 3, _params(), refresh=True) == {
        "pass_order": 2, "graph": 0, "merge_halves": 1, "fuse_steps": 1}
    # a plane-wave grid (one pass per step) never fuses; a long tau axis may
    calls.clear()
    autotune.tune(1, 1, 256, 2, _params(), refresh=True)
    assert all(c["fuse_steps"] == 0 for c in calls)
    calls.clear()
    autotune.tune(8, 8, 1024, 2, _params(), refresh=True)
    assert {c["fuse_steps"] for c in calls} == {0, 1}


def test_tuner_keeps_literal_half_steps_where_merging_is_refused(fake_tuner):
    """A dk profile or a transverse map keeps the literal N/2 - L - N/2 (the
    plan refuses merge_halves there), and so does merge_halves=False."""
    import numpy as np
    calls = fake_tuner({(1, 0): 0.5})
    prof = brahms.Params(dz=0.01, fields=[brahms.FieldParams(kappa=1.0)] * 2, dk=np.ones(10))
    assert autotune.tune(8, 8, 8, 2, prof)["merge_halves"] == 0
    mapped = brahms.Params(dz=0.01, fields=[brahms.FieldParams(kappa=1.0)] * 2,
                           dk_map=np.ones((8, 8)))
    assert autotune.tune(8, 8, 8, 2, mapped)["merge_halves"] == 0
    assert autotune.tune(8, 8, 8, 2, _params(), merge_halves=False)["merge_halves"] == 0
    assert all(c["merge_halves"] == 0 and c["fuse_steps"] == 0 for c in calls)


def test_bench_refuses_more_than_one_gpu():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode != 0
    assert "one GPU" in (res.stdout + res.stderr)
