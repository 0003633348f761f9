"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle's C hop (built with gcc) and the library's host layer (tm_api.cpp
rebuilt with host-side sanitizers and linked with the already built kernel
objects), each driven by a small program in tests/sanitize/."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.slow
def test_oracle_hop_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-o", exe, os.path.join(ROOT, "oracle", "tm_oracle.c"), os.path.join(HERE, "oracle_driver.c"), "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "0 failures" in r.stdout


@pytest.mark.slow
def test_host_layer_under_sanitizers(tmp_path):
    from paper_1311_4462_amd import build as B
    objs = [o for o in glob.glob(os.path.join(B.OBJDIR, "*.o")) if not o.endswith("tm_api.cpp.o")]
    if len(objs) < len(B.SOURCES) - 1:
        pytest.skip("kernel objects not built (run __graft_entry__.build())")
    hipcc = B._hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    api_o = str(tmp_path / "tm_api_san.o")
    _run([hipcc, *B.FLAGS, "-O1", "-g", *san, "-c", os.path.join(B.CSRC, "tm_api.cpp"), "-o", api_o])
    lib = str(tmp_path / "libtm_san.so")
    _run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *san, "-o", lib, api_o, *objs,
          "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    drv_o = str(tmp_path / "abi_driver.o")
    _run([hipcc, "-O1", "-g", *san, f"-I{B.INCLUDE}", "-c", os.path.join(HERE, "abi_driver.cpp"), "-o", drv_o])
    exe = str(tmp_path / "abi_driver")
    _run([hipcc, *san, "-o", exe, drv_o, f"-L{tmp_path}", "-ltm_san", f"-Wl,-rpath,{tmp_path}"])
    r = _run([exe], env=ENV, timeout=300)
    assert "0 failures" in r.stdout
