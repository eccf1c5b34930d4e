"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU:

* the oracle's C routines (oracle/oracle_sum.c, gcc) driven by
  tests/sanitize/oracle_harness.c over empty, special and random inputs;
* the library's host code (validation, error messages, plan tables, the
  tuner's candidate search, probe formulas, the no-device path, shutdown):
  runtime.hip and probes.hip built with host-only sanitizers, linked with
  the library's other objects, driven by tests/sanitize/abi_harness.cpp
  with no GPU present.

(The lane-level emulation of the segmented kernel runs under the same
sanitizers in test_seg_runs_emulation.py.)"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2004_05371_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2004_05371_amd", "_build")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_routines_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_harness")
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-o", exe, os.path.join(HERE, "oracle_harness.c"),
                    os.path.join(ROOT, "oracle", "oracle_sum.c"), "-lm"], check=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=SAN_ENV)
    assert p.returncode == 0 and "oracle harness ok" in p.stdout, p.stderr[-3000:]


HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)), reason="needs the ROCm compilers")
@pytest.mark.skipif(_has_gpu(), reason="drives the no-device path")
def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2004_05371_amd import build as B
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-fno-gpu-flush-denormals-to-zero", "-Wno-unused-command-line-argument",
              "-Wno-pass-failed"]
    # host-only sanitizers: each -fsanitize= applies to the host pass only
    host_san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    procs, objs = [], []
    for src in ("runtime", "probes"):
        obj = str(tmp_path / (src + ".san.o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *common, *host_san, "-c", os.path.join(CSRC, src + ".hip"), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for src in ("reduce", "segmented", "stencil"):  # the kernels' objects, as the library build makes them
        obj = os.path.join(BUILD, src + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(os.path.join(CSRC, src + ".hip")):
            os.makedirs(BUILD, exist_ok=True)
            B._compile(src + ".hip")
        objs.append(obj)
    for pr in procs:
        out, err = pr.communicate(timeout=600)
        assert pr.returncode == 0, err[-3000:]
    lib = str(tmp_path / "libredsum_san.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs], check=True,
                   capture_output=True)
    exe = str(tmp_path / "abi_harness")
    subprocess.run([CLANGXX, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I" + os.path.join(ROOT, "include"), "-o", exe, os.path.join(HERE, "abi_harness.cpp"),
                    "-L" + str(tmp_path), "-lredsum_san", "-Wl,-rpath," + str(tmp_path)], check=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=SAN_ENV)
    assert p.returncode == 0 and "abi harness ok" in p.stdout, (p.stdout[-2000:], p.stderr[-3000:])
