"""Build libfcmp.so in-tree with hipcc for gfx950.

    python -m paper_1205_4139_amd.build        (or: python paper_1205_4139_amd/build.py)

Every HIP and host source under csrc/ is compiled to an object with
``hipcc --offload-arch=gfx950 -O3`` and linked into
``paper_1205_4139_amd/libfcmp.so``.  Floating-point policy: no fast-math;
FMA contraction allowed (``-ffp-contract=fast``); packed FP32 instructions
disabled (``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libfcmp.so")
BUILD = os.path.join(HERE, "_build")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-ffp-contract=fast",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip") or name.endswith(".cpp"):
            out.append(os.path.join(CSRC, name))
    return out


# Host-only sanitizer builds (CPU tests): the host code of every source is
# instrumented, the device code is not; the runtime is preloaded into the
# test process (sanitizer_runtime), so the library links without it.
SANITIZERS = {
    "address": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"],
    "undefined": ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
                  "-fno-sanitize-recover=undefined"],
}


def sanitizer_runtime(kind: str) -> str:
    """Path of the clang runtime to preload for a sanitizer build."""
    name = {"address": "libclang_rt.asan-x86_64.so",
            "undefined": "libclang_rt.ubsan_standalone-x86_64.so"}[kind]
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang")
    for cand in (clang, "/opt/rocm/llvm/bin/clang"):
        if os.path.exists(cand):
            r = subprocess.run([cand, f"-print-file-name={name}"], capture_output=True, text=True)
            if r.returncode == 0 and os.path.exists(r.stdout.strip()):
                return r.stdout.strip()
    raise RuntimeError(f"{name} not found")


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [hipcc()] + FLAGS + list(extra) + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: str = "") -> str:
    """Compiles libfcmp.so; with sanitize ("address" or "undefined") a
    host-instrumented copy paper_1205_4139_amd/_build_<kind>/libfcmp.so."""
    build_dir = BUILD if not sanitize else os.path.join(HERE, f"_build_{sanitize}")
    out = OUT if not sanitize else os.path.join(build_dir, "libfcmp.so")
    extra = SANITIZERS[sanitize] if sanitize else []
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", "8"))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, extra), srcs))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
