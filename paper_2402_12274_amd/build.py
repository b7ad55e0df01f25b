"""Build libmdt.so (host C++ + gfx950 HIP kernels) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmdt.so")
LOADGEN = os.path.join(HERE, "libmdt_loadgen.so")

# (source, extra defines): the batch kernel variants compile once per launch
# policy and direction
SOURCES = [(s, ()) for s in ("types.cpp", "compile.cpp", "api.cpp", "requests.cpp", "device.hip", "batch.hip",
                             "server.cpp", "trace.cpp")]
SOURCES += [("batch_variants.hip", (f"MDT_BATCH_POLICY={p}", f"MDT_BATCH_UNPACK={u}")) for p in (0, 1, 2)
            for u in (0, 1)]
ARCH = os.environ.get("MDT_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include")]
HIP_ONLY = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _newest_header() -> float:
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    heads += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(h) for h in heads)


def _compile(item) -> str:
    src, defines = item if isinstance(item, tuple) else (item, ())
    path = os.path.join(CSRC, src)
    tag = "".join("_" + d.split("=")[1] for d in defines)
    obj = os.path.join(BUILD, src.replace(".", "_") + tag + ".o")
    # MDT_BUILD_INCREMENTAL=1 (development): keep an object newer than its
    # source and every header; the default rebuilds everything
    if os.environ.get("MDT_BUILD_INCREMENTAL") == "1" and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(path), _newest_header()):
        return obj
    cmd = ["hipcc", *COMMON, *[f"-D{d}" for d in defines]]
    if src.endswith(".hip"):
        cmd += HIP_ONLY
    cmd += ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s[0]))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread", "-ldl"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    # open-loop load generator for the serving benchmark (public C ABI only)
    lg_obj = _compile("loadgen.cpp")
    tmp = LOADGEN + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "-o", tmp, lg_obj, LIB, "-Wl,-rpath,$ORIGIN", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LOADGEN)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
