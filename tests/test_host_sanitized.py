"""The host side of libevp.so (argument checks, workspace layout and guard regions, error
strings) under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU: evp_api.cpp is
rebuilt with the sanitizers on its host code only and linked with the kernel objects of the normal
build; a child process preloads the sanitizer runtime and runs the host-only ABI tests against it.
Any out-of-bounds access or undefined behaviour in the host code fails the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1803_09563_amd")
CLANG = "/opt/rocm/llvm/bin/clang"


def _runtime():
    r = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                       text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_host_library_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, PKG)
    import build as B
    sys.path.pop(0)
    rt = _runtime()
    assert rt, "the ROCm clang sanitizer runtime is missing"
    kernels = [s for s in B.SOURCES if s.endswith(".hip")]
    objs = [os.path.join(B.OBJDIR, os.path.splitext(s)[0] + ".o") for s in kernels]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
    api = str(tmp_path / "evp_api_san.o")
    subprocess.run([B.HIPCC, *B.COMMON, *san, "-x", "hip", "-c", os.path.join(B.CSRC, "evp_api.cpp"),
                    "-o", api], check=True, capture_output=True)
    lib = str(tmp_path / "libevp_san.so")
    subprocess.run([B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", *san, *objs, api, "-o", lib],
                   check=True, capture_output=True)
    env = dict(os.environ)
    # the sanitizer runtime must come first; anything already preloaded stays after it
    env["LD_PRELOAD"] = rt + (" " + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env.update(EVP_LIB=lib, ASAN_OPTIONS="detect_leaks=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = ("import ctypes, os, paper_1803_09563_amd as e; "
             "assert e.LIB_PATH == os.environ['EVP_LIB']; "
             "assert hasattr(ctypes.CDLL(None), '__asan_init'); "
             "assert e.workspace_bytes(64, 48, 32, walls=True) > 0; print('sanitized host library loaded')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "sanitized host library loaded" in r.stdout, (r.stdout + r.stderr)[-4000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_abi.py"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
