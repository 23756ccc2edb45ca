"""AddressSanitizer and UndefinedBehaviorSanitizer builds, on the CPU: the
FP64 oracle (every entry point, each dynamics family, both obstacle terms,
sub-rollouts, the control terms) and the host side of the C ABI (validation,
workspace and layout arithmetic, the batched work list; no device work).
Each build runs a driver that exits non-zero on the first report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests")
CSRC = os.path.join(ROOT, "paper_1503_00330_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _gpu_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-6000:])
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(HERE, "sanitize_oracle.c"), "-o", exe, "-lm"], str(tmp_path))
    r = _run([exe], str(tmp_path))
    assert r.stdout.strip().endswith("ok")


@pytest.mark.skipif(_gpu_visible(), reason="the driver passes fake device pointers; CPU only")
@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_c_abi_host_code_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clangxx = "/opt/rocm/llvm/bin/clang++"
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
             "-mllvm", "-amdgpu-mfma-vgpr-form=1",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    procs, objs = [], []
    for src in ("capi", "direct", "mfma", "adjoint"):
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc] + flags + ["-c", os.path.join(CSRC, src + ".hip"), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, err[-4000:]
    drv = str(tmp_path / "drv.o")
    _run([clangxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-c", os.path.join(HERE, "sanitize_abi.cpp"),
          "-o", drv], str(tmp_path))
    exe = str(tmp_path / "abi_san")
    _run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined"] + objs + [drv, "-o", exe], str(tmp_path))
    r = _run([exe], str(tmp_path))
    assert r.stdout.strip().endswith("ok")
