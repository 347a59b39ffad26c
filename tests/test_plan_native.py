"""The host planner and its plan-table checks built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host code only, no device code) and driven over the ragged
recipe's draws and the mixed geometries of the plan tests, for every op (CPU only)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_02401_amd", "csrc")
MIXED = [((128, 256), 2, 4, 0.5), ((64, 64, 64), 4, 3, 1.0), ((512,), 8, 5, 2.0), ((256, 128), 8, 4, 1.5),
         ((96, 160), 3, 3, 1.0), ((32, 32, 16), 6, 2, 0.5), ((1024,), 1, 7, 1.0), ((64, 64), 4, 1, 1.0),
         ((16, 16), 8, 4, 1.0), ((128, 128), 2, 0, 1.0)]


def _plan_text(op, descs):
    lines = [f"plan {op} {len(descs)}"]
    for shape, order, levels, s in descs:
        sh = list(shape) + [1] * (3 - len(shape))
        lines.append(f"{len(shape)} {sh[0]} {sh[1]} {sh[2]} {order} {levels} {s!r}")
    return "\n".join(lines) + "\n"


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are missing")
    out = str(tmp_path_factory.mktemp("native") / "plan_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "filters.cpp"),
           os.path.join(ROOT, "tests", "native", "plan_check.cpp"),
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _run(checker, text, persistent="0"):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               ESWAVE_PLAN_PERSISTENT=persistent)
    r = subprocess.run([checker], input=text, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.stdout[-2000:], r.stderr[-6000:])
    return r.stdout.split()


def test_mixed_every_op(checker):
    text = "".join(_plan_text(op, MIXED) for op in range(4))
    out = _run(checker, text)
    assert int(out[1]) == 4 and int(out[2]) > 0


@pytest.mark.parametrize("persistent", ["0", "1"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ragged_recipe_draws(checker, seed, persistent):
    descs = list(inputs.ragged_descriptors(200, seed))
    text = "".join(_plan_text(op, descs) for op in range(4))
    out = _run(checker, text, persistent)
    assert int(out[1]) == 4


def test_random_small_plans(checker):
    """Random geometries: 1-3 D, every order, depths up to the largest the sides allow, odd
    multiples of 2^levels, one to six instances per plan."""
    gen = np.random.default_rng(123)
    text = ""
    for _ in range(60):
        descs = []
        for _ in range(int(gen.integers(1, 7))):
            d = int(gen.integers(1, 4))
            levels = int(gen.integers(0, 6))
            shape = tuple(int(gen.integers(1, 6 if d == 3 else 12)) * (1 << levels) for _ in range(d))
            descs.append((shape, int(gen.integers(1, 9)), levels, float(gen.choice([-1.0, 0.5, 1.5]))))
        text += _plan_text(int(gen.integers(0, 4)), descs)
    for persistent in ("0", "1"):
        out = _run(checker, text, persistent)
        assert int(out[1]) == 60
