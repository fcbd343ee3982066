"""Host code of the serving scheduler under sanitizers (CPU only, fake
backend): AddressSanitizer + UndefinedBehaviorSanitizer on randomized
single-threaded sequences and on concurrent submitters / scheduler /
releaser threads, and ThreadSanitizer on the concurrent run.  The
sanitizers instrument host code only; device code is compiled as usual and
never runs here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2209_08241_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("bn_serve.hip", "bn_batch.hip", "bn_capi.hip",
                                           "bn_kernels.hip", "bn_autotune.hip",
                                           "bn_workspace.hip")]
DRIVER = os.path.join(ROOT, "tests", "native", "serve_fake_stress.cpp")
HIPCC = "/opt/rocm/bin/hipcc"
BASE = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
SAN = {
    "asan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
             "-fno-omit-frame-pointer"],
    "tsan": ["-Xarch_host", "-fsanitize=thread"],
}

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    out = {}
    for name, flags in SAN.items():
        exe = str(d / f"stress_{name}")
        res = subprocess.run([HIPCC, *BASE, *flags, *SOURCES, DRIVER, "-o", exe],
                             stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert res.returncode == 0, res.stdout[-3000:]
        out[name] = exe
    yield out
    shutil.rmtree(d, ignore_errors=True)


def run(exe, mode, env_extra):
    env = dict(os.environ, **env_extra)
    res = subprocess.run([exe, mode], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                         env=env, timeout=600)
    assert res.returncode == 0 and f"ok {mode}" in res.stdout, res.stdout[-4000:]
    assert "runtime error" not in res.stdout and "WARNING: ThreadSanitizer" not in res.stdout, \
        res.stdout[-4000:]


@pytest.mark.parametrize("mode", ["single", "threads"])
def test_asan_ubsan(binaries, mode):
    run(binaries["asan"], mode, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
                                 "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})


def test_tsan(binaries):
    run(binaries["tsan"], "threads", {"TSAN_OPTIONS": "halt_on_error=1"})
