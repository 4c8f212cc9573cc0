"""Build libpathgraph.so from csrc/*.hip with hipcc for gfx950 (in-tree)."""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC_DIR = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "_lib")
OBJ_DIR = os.path.join(HERE, "_build")
SANITIZE = os.environ.get("PG_SANITIZE") == "1"
LIB_PATH = os.path.join(LIB_DIR, "libpathgraph_san.so" if SANITIZE else "libpathgraph.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# PG_SANITIZE=1: AddressSanitizer + UndefinedBehaviorSanitizer on the host
# code only (argument validation, workspace carving, launch order); the
# device code is built as usual.  The runtime comes from LD_PRELOAD.
HOST_SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build(verbose: bool = False, jobs: int = 8, sanitize: bool | None = None) -> str:
    """Compile every csrc/*.hip to an object and link the shared library
    (with ``sanitize``, default PG_SANITIZE=1: the host-sanitized
    libpathgraph_san.so)."""
    sanitize = SANITIZE if sanitize is None else sanitize
    os.makedirs(LIB_DIR, exist_ok=True)
    obj_dir = OBJ_DIR + ("_san" if sanitize else "")
    os.makedirs(obj_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(SRC_DIR, "*.hip")))
    out = os.path.join(LIB_DIR, "libpathgraph_san.so" if sanitize else "libpathgraph.so")

    def compile_one(src):
        obj = os.path.join(obj_dir, os.path.basename(src)[:-4] + ".o")
        cmd = [HIPCC, *FLAGS, *(HOST_SAN if sanitize else []), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msgs = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                         if "packed-fp32-ops' is not a recognized feature" not in line)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
        if msgs.strip() and verbose:
            print(msgs)
        return obj

    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, out)
    return out
