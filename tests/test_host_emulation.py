"""The engine's host code and kernels run on the CPU under AddressSanitizer
and UndefinedBehaviorSanitizer (tests/hostemu: the HIP runtime emulated,
kernels executed block by block with fibers as threads), through the call
sequences of the batch and plan tests: every batch create / schedule / bind /
run / destroy sequence, long tau axes in batches, reduced dimensions, the
autotuner's sequence of rebinds, graph replays.  Each pass and table launch
is checked before it runs: every range its arguments let a block touch lies
in the fields or workspace of its own problem.  Batch members must come out
bitwise equal to the same problem run alone (as on the GPU).

A second build of batch.hip ("variant") captures its graphs with parallel
branches and accepts fused step pairs in batches that hold long tau
problems, the two configurations that are switched off in the library; it
runs the batch sequences too.

The build (clang++, host only, a few minutes on a cold cache) is kept under
tests/hostemu/_build, keyed by a hash of the sources."""
import concurrent.futures
import hashlib
import os
import shutil
import subprocess

import pytest

from paper_2609_08384_amd.build import SOURCES as LIB_SOURCES

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "hostemu")
CSRC = os.path.join(ROOT, "paper_2609_08384_amd", "csrc")
SCENARIOS = ["plain_batches", "merged_batches", "long_tau_batches", "long_tau_fused", "three_field",
             "reduced_dims", "tuner_sequence", "plans", "three_lengths", "stream_graphs", "splits"]
VARIANT_SCENARIOS = ["plain_batches", "merged_batches", "long_tau_batches", "long_tau_fused",
                     "three_field", "reduced_dims", "tuner_sequence"]

# text of batch.hip changed for the variant build (each must be present)
_BRANCHES = ("constexpr bool kParallelBranches = false;", "constexpr bool kParallelBranches = true;")
_LONG_TAU_REFUSAL = ('''  if (fuse_steps)
    for (brahms_plan p : b->plans)
      if (brahms::detail::long_tau(*p))
        return fail(BRAHMS_E_UNSUPPORTED, "fuse_steps in a batch with a long tau problem");''', "")


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def _flags():
    return ["-x", "c++", "-std=c++17", "-O1", "-g0", "-fsanitize=address,undefined",
            "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
            "-I" + EMU, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
            "-Wno-unused-function", "-Wno-unused-variable"]


def _source_hash():
    h = hashlib.sha256()
    files = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))]
    files += [os.path.join(ROOT, "include", "brahms.h")]
    files += [os.path.join(EMU, f) for f in ("emu.cpp", "emu.hpp", "drive.cpp")]
    files += [os.path.join(EMU, "hip", "hip_runtime.h")]
    for f in files:
        h.update(f.encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(_flags()).encode())
    h.update(repr((_BRANCHES, _LONG_TAU_REFUSAL)).encode())
    return h.hexdigest()[:16]


def _variant_source(out):
    src = open(os.path.join(CSRC, "batch.hip")).read()
    for old, new in (_BRANCHES, _LONG_TAU_REFUSAL):
        assert old in src, "batch.hip changed: update the variant build of the host emulation"
        src = src.replace(old, new)
    path = os.path.join(out, "batch_variant.hip")
    with open(path, "w") as fh:
        fh.write(src.replace('"../../include/brahms.h"', '"brahms.h"'))
    return path


def _build(out):
    cxx = _clang()
    os.makedirs(out, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in LIB_SOURCES]
    srcs += [_variant_source(out), os.path.join(EMU, "emu.cpp"), os.path.join(EMU, "drive.cpp")]

    def compile_one(src):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        r = subprocess.run([cxx, *_flags(), "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
        objs = dict(zip([os.path.basename(s) for s in srcs], ex.map(compile_one, srcs)))
    common = [objs[k] for k in ["emu.cpp", "drive.cpp"] + [s for s in LIB_SOURCES if s != "batch.hip"]]
    exes = {}
    for name, batch in (("drive", "batch.hip"), ("drive_variant", "batch_variant.hip")):
        exe = os.path.join(out, name)
        r = subprocess.run([cxx, "-fsanitize=address,undefined", "-o", exe + ".tmp", *common, objs[batch]],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        os.replace(exe + ".tmp", exe)
        exes[name] = exe
    return exes


@pytest.fixture(scope="module")
def runs():
    if _clang() is None:
        pytest.skip("clang++ not available")
    out = os.path.join(EMU, "_build", _source_hash())
    exes = {n: os.path.join(out, n) for n in ("drive", "drive_variant")}
    if not all(os.path.exists(e) for e in exes.values()):
        exes = _build(out)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:detect_stack_use_after_return=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    jobs = [("drive", s) for s in SCENARIOS] + [("drive_variant", s) for s in VARIANT_SCENARIOS]

    def run(job):
        r = subprocess.run([exes[job[0]], job[1]], capture_output=True, text=True, env=env, timeout=1800)
        return job, r

    with concurrent.futures.ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        return dict(ex.map(run, jobs))


def _check(r):
    tail = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, tail
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, tail
    assert "checked passes" in r.stdout, tail


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_engine_under_sanitizers(runs, scenario):
    _check(runs[("drive", scenario)])


@pytest.mark.parametrize("scenario", VARIANT_SCENARIOS)
def test_branched_graph_variant_under_sanitizers(runs, scenario):
    r = runs[("drive_variant", scenario)]
    _check(r)
    if scenario == "long_tau_fused":
        assert "long tau fused batches group_max=1: ok" in r.stdout
