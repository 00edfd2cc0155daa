"""Build liblbm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2010_01628_amd.build

Every HIP translation unit is compiled with packed-FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "liblbm.so")
BUILD_DIR = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse a*b+c only inside one source expression, so every kernel that
    # inlines the collision rounds it identically (A-B and AA agree bitwise)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


# host-side AddressSanitizer + UndefinedBehaviorSanitizer for the C-ABI layer;
# every flag goes to the host pass only (GPU code is never built with them)
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, extra=(), obj: str | None = None) -> str:
    obj = obj or os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + list(extra) + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


def build_host_sanitized(out: str) -> str:
    """The same library with its host code (the C ABI: parameter checks,
    handle management, launch set-up) under ASan and UBSan, for CPU tests of
    the error paths.  The kernels' objects are the ordinary ones; load the
    result with clang's ASan runtime preloaded (``asan_runtime()``)."""
    os.makedirs(os.path.join(BUILD_DIR, "san"), exist_ok=True)
    newest = max(os.path.getmtime(p) for p in glob.glob(os.path.join(CSRC, "*")))
    jobs = []
    for src in sources():
        if src.endswith(".cpp"):
            obj = os.path.join(BUILD_DIR, "san", os.path.basename(src) + ".o")
            jobs.append((src, HOST_SANITIZE + ["-g"], obj))
        else:
            obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
            if not os.path.exists(obj) or os.path.getmtime(obj) < newest:
                jobs.append((src, (), obj))
            else:
                jobs.append((None, None, obj))
    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(lambda j: _compile(*j) if j[0] else j[2], jobs))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-shared-libasan"] + HOST_SANITIZE[:4] + \
        ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


def asan_runtime() -> str:
    """Path of the clang ASan runtime that the sanitized library links."""
    r = subprocess.run([HIPCC, "--offload-arch=" + ARCH, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else ""
    if not os.path.isabs(path) or not os.path.exists(path):
        cand = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not cand:
            raise FileNotFoundError("clang ASan runtime not found")
        path = cand[0]
    return path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
