"""Build the gfx950 HIP library librkmips.so in-tree (hipcc, one object per source)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(OUT_DIR, "librkmips.so")
SOURCES = ["k_prep.hip", "k_topk.hip", "k_refine.hip", "k_cone.hip", "k_saalsh.hip", "k_query.hip", "k_saalsh_query.hip",
           "k_diag.hip", "api.cpp", "query.cpp", "serve.cpp", "mem.cpp", "persist.cpp"]
ARCH = os.environ.get("RKMIPS_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-fno-gpu-rdc",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         "-Wno-unused-but-set-variable"]


def _sources():
    return [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


LIB_SAN = os.path.join(OUT_DIR, "librkmips_san.so")
# host code only: each sanitizer flag applies to the host compilation (the device code of
# the .hip objects is the same as in the plain build)
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g"]


def build_sanitized(jobs: int = 8) -> str:
    """librkmips_san.so: the host-only sources (.cpp: the C ABI, index files, batching,
    serving, memory) with AddressSanitizer and UndefinedBehaviorSanitizer, linked with the
    plain build's kernel objects.  Load it with the clang ASan runtime preloaded."""
    objdir = os.path.join(OUT_DIR, "obj")
    sandir = os.path.join(OUT_DIR, "obj_san")
    os.makedirs(sandir, exist_ok=True)
    srcs = _sources()
    hip_objs = [os.path.join(objdir, s.rsplit(".", 1)[0] + ".o") for s in srcs if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in hip_objs):
        build()

    def compile_one(src):
        obj = os.path.join(sandir, src.rsplit(".", 1)[0] + ".o")
        cmd = ["hipcc", *FLAGS, *SAN_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        cpp_objs = list(ex.map(compile_one, [s for s in srcs if s.endswith(".cpp")]))
    tmp = LIB_SAN + f".tmp{os.getpid()}"
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-o", tmp, *hip_objs, *cpp_objs])
    os.replace(tmp, LIB_SAN)
    return LIB_SAN


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime that librkmips_san.so needs preloaded."""
    out = subprocess.run(["hipcc", "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True).stdout.strip()
    return out


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source for gfx950 and link librkmips.so (always recompiles)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    objdir = os.path.join(OUT_DIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    srcs = _sources()

    def compile_one(src):
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        cmd = ["hipcc", *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{err}")
        if verbose and err.strip():
            print(err, file=sys.stderr)
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
