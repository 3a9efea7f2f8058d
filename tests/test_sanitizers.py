"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's host code (builder, serving rules, CPU matcher, C-ABI argument
checks) is rebuilt with ``-Xarch_host -fsanitize=address,undefined`` (the
device code is compiled as usual and never runs here), the C oracle with
clang's ASan/UBSan, and the GPU-free tests are run against both builds in a
child process with the ASan runtime preloaded.  Any heap overflow, use after
free or undefined behaviour aborts the child and fails this test.
"""

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
CLANG = os.path.join(ROCM, "lib", "llvm", "bin", "clang")
ASAN_RT = sorted(glob.glob(os.path.join(ROCM, "lib", "llvm", "lib", "clang", "*", "lib", "linux",
                                        "libclang_rt.asan-x86_64.so")))
HOST_TESTS = ["tests/test_builder.py", "tests/test_serve_host.py", "tests/test_host_match.py",
              "tests/test_oracle.py"]


@pytest.mark.skipif(not ASAN_RT or not os.path.exists(CLANG) or shutil.which("gcc") is None,
                    reason="clang's AddressSanitizer runtime is not installed")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as oracle_build
    from paper_1412_7789_amd import build as lib_build

    lib = lib_build.build(out=str(tmp_path / "libpfac.so"), sanitize=True, objdir=str(tmp_path / "obj"))
    ora = oracle_build.build(out=str(tmp_path / "libacoracle.so"), cc=CLANG,
                             extra=("-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                                    "-fno-sanitize-recover=undefined", "-shared-libasan"))
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": ASAN_RT[-1],
        # CPython itself is not instrumented and keeps objects alive at exit
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "PFAC_LIBRARY": lib,
        "ORACLE_LIBRARY": ora,
        # the HIP runtime is all the host tests need; torch is not loaded
        "PFAC_NO_TORCH": "1",
    })
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider", *HOST_TESTS]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    # the sanitized builds were the ones loaded
    probe = ("import sys; from paper_1412_7789_amd import _lib; from oracle import load_library; "
             "_lib.load(); load_library(); "
             "m = open('/proc/self/maps').read(); "
             "sys.exit(0 if sys.argv[1] in m and sys.argv[2] in m and 'torch' not in sys.modules else 1)")
    res = subprocess.run([sys.executable, "-c", probe, lib, ora], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
