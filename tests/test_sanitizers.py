"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C source (plain and OpenMP builds) and the library's host code (device code
built as usual but never run here) are compiled with -fsanitize=address,undefined and
driven by the small C programs in tests/sanitize/: every oracle function on small ragged
boxes, and every C-ABI entry point that needs no device work, including the failure path
of context creation.  Any sanitizer report, or a leak at exit, fails the run."""
import concurrent.futures
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ENV = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe, env=ENV):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.parametrize("openmp", [False, True])
def test_oracle_under_sanitizers(tmp_path, openmp):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    exe = str(tmp_path / "oracle_driver")
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True)
    out = _run(exe, dict(ENV, OMP_NUM_THREADS="4"))
    assert out.strip().endswith("oracle driver ok")


@pytest.mark.slow
def test_abi_host_code_under_sanitizers(tmp_path):
    from paper_1204_2088_amd import build as B
    hipcc = B.hipcc()
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
    if not (shutil.which(hipcc) or os.path.exists(hipcc)) or not os.path.exists(clang):
        pytest.skip("no ROCm compilers")
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs, cmds = [], []
    for src in B.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([hipcc, "-O1", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}", *san, "-Xclang",
                     "-target-feature", "-Xclang", "-packed-fp32-ops", "-w", "-I", B.INCLUDE, "-I", B.CSRC, "-c",
                     os.path.join(B.CSRC, src), "-o", obj])
    jobs = max(1, min(len(cmds), os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(subprocess.run, c, check=True) for c in cmds]:
            f.result()
    drv = str(tmp_path / "abi_driver.o")
    subprocess.run([clang, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", B.INCLUDE, "-c", os.path.join(HERE, "sanitize", "abi_driver.c"), "-o", drv], check=True)
    exe = str(tmp_path / "abi_driver")
    subprocess.run([hipcc, "-fsanitize=address,undefined", "-fno-gpu-sanitize", f"--offload-arch={B.ARCH}", "-o", exe,
                    drv, *objs], check=True)
    out = _run(exe)
    assert out.strip().endswith("abi driver ok")
