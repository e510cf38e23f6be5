"""The host side of the C-ABI under the address and undefined-behaviour
sanitizers (CPU only): `rswr_host.cpp` is compiled with the sanitizers on its
host code, linked with `tests/host/plan_fuzz.cpp`, and run over thousands of
seeded descriptors (uniform and explicit windows, every built tile shape,
FIXED and QUIET spans, interior sources, the one-launch waits, and requests
that must be refused).  Any heap or stack error, undefined shift or overflow
aborts the run; the driver also checks the decomposition of Sec. 2.2 /
Sec. 3 (Eq. (4) order, Eq. (15) ownership) and that every owned node is
stored by exactly one tile.  The kernels are taken from the built library
(the driver never launches one)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2203_10477_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "lib", "llvm", "bin", "clang++")
SAN = ["address", "undefined"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.slow
def test_plan_logic_under_address_and_ub_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not installed")
    if not os.path.exists(os.path.join(PKG, "librswr.so")):
        pytest.skip("librswr.so not built")
    host_o = str(tmp_path / "host.o")
    drv_o = str(tmp_path / "drv.o")
    exe = str(tmp_path / "plan_fuzz")
    # sanitizers on the host pass only (the device pass of the same file is
    # built as usual)
    host_san = []
    for s in SAN:
        host_san += ["-Xarch_host", "-fsanitize=" + s]
    host_san += ["-Xarch_host", "-fno-sanitize-recover=undefined"]
    _run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer",
          "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          *host_san, "-c", os.path.join(PKG, "csrc", "rswr_host.cpp"), "-o", host_o])
    cpu_san = ["-fsanitize=" + ",".join(SAN), "-fno-sanitize-recover=undefined"]
    _run([CLANG, "-O1", "-g", "-std=c++17", *cpu_san, "-c",
          os.path.join(ROOT, "tests", "host", "plan_fuzz.cpp"), "-o", drv_o])
    _run([CLANG, *cpu_san, drv_o, host_o, "-L" + PKG, "-lrswr", "-L" + os.path.join(ROCM, "lib"),
          "-lamdhip64", "-Wl,-rpath," + PKG, "-Wl,-rpath," + os.path.join(ROCM, "lib"),
          "-o", exe])
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = _run([exe, "3000"], env=env, timeout=300)
    line = r.stdout.strip().splitlines()[-1]
    made, refused = int(line.split()[1]), int(line.split()[3])
    assert line.endswith("failures 0"), line
    assert made > 1000 and refused > 500, line
