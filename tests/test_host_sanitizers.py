"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer
and under ThreadSanitizer, on the CPU.

Every source of the library is compiled with the sanitizers on its host side
only (the device code is built as usual and never runs here), and linked with
the C program in tests/host_sanitize/host_checks.c, which exercises:
  - the argument validation and error paths of the C ABI;
  - the checkpoint parser on random, cut, misaligned and plausible-looking
    images, all of which must be refused;
  - the host gate builder (Eq. (1) split into three-site terms, diagonalised
    and exponentiated in FP64) from six threads at once;
  - the serving scheduler: twelve requests admitted by footprint with three
    slots, each on its own thread; without a GPU every request fails at its
    first device allocation, so the admission loop, the condition variable
    and the per-request error paths all run concurrently.
A sanitizer report makes the program exit non-zero, and the test fails with it.
On a machine with a GPU the same program would also run the device paths; the
test is meant for the CPU-only suite and is skipped when a GPU is visible.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2401_05301_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def _gpu_visible():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def _build(tmp, kind):
    """Objects of every library source plus the check program, linked into one
    executable; `kind` is "address+undefined" or "thread"."""
    sans = kind.split("+")
    host_flags = []
    for s in sans:
        host_flags += ["-Xarch_host", "-fsanitize=" + s]
    common = ["-O1", "-g", "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include")]
    objs, procs = [], []
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith((".hip", ".cpp")):
            continue
        obj = os.path.join(tmp, f.split(".")[0] + ".o")
        cmd = [HIPCC, "--offload-arch=gfx950", "-x", "hip", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + common + host_flags + \
              ["-c", os.path.join(CSRC, f), "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out[-3000:]
    drv = os.path.join(tmp, "host_checks.o")
    subprocess.run([HIPCC, "-x", "c"] + common + host_flags +
                   ["-c", os.path.join(HERE, "host_sanitize", "host_checks.c"), "-o", drv],
                   check=True, capture_output=True, timeout=300)
    exe = os.path.join(tmp, "host_checks")
    link = [CLANG] + ["-fsanitize=" + s for s in sans] + objs + [drv, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib",
                                                                "-lamdhip64", "-lpthread", "-o", exe]
    r = subprocess.run(link, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kind", ["address+undefined", "thread"])
def test_host_code_under_sanitizers(tmp_path, kind):
    if not os.path.exists(CLANG) or not os.path.exists(HIPCC):
        pytest.skip("ROCm clang toolchain not found")
    if _gpu_visible():
        pytest.skip("CPU-only check (device paths are covered by the GPU tests)")
    exe = _build(str(tmp_path), kind)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "host checks: ok" in r.stdout, report
    for word in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer"):
        assert word not in r.stderr, report
