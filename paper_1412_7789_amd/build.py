"""Compile the HIP library ``libpfac.so`` for gfx950 with hipcc (in-tree).

Every call recompiles; ``python -m paper_1412_7789_amd.build`` does the same
from the shell.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpfac.so")
# the filtered kernels of each stride compile in their own unit, in parallel
SOURCES = ["filtered_s1k1.hip", "filtered_s1k2.hip", "filtered_s1k3.hip", "filtered_s2.hip", "filtered_s4.hip",
           "kernels.hip", "plan.cpp", "capi.cpp", "serve.cpp", "host_match.cpp"]
ARCH = os.environ.get("PFAC_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the CPU test
# leg: every flag reaches the host compiler only, the device code is built as
# usual, and the runtime is linked as a shared library (preloaded by the test).
SANITIZE_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SANITIZE_LINK_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                       "-Xarch_host", "-shared-libasan"]


def build(out: str = LIB, verbose: bool = False, sanitize: bool = False, objdir: str = "") -> str:
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    objdir = objdir or os.path.join(HERE, "_build_sanitize" if sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    extra = SANITIZE_HOST_FLAGS if sanitize else []

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, *extra, f"-I{INCLUDE}", f"-I{CSRC}", "-x", "hip", "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
        warn = "\n".join(l for l in (res.stderr or "").splitlines()
                         if "packed-fp32-ops" not in l and "target-feature" not in l
                         and l.strip() and "warning generated" not in l)
        if verbose and warn:
            print(warn, file=sys.stderr)
        return obj

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *(SANITIZE_LINK_FLAGS if sanitize else []),
           *objs, "-o", tmp, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True), file=sys.stderr)
