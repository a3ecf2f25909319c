"""Build libnmf.so (HIP for gfx950) in-tree with hipcc, and the probes/ programs.

    python -m paper_1009_0881_amd.build [--jobs N] [--debug]

Every call recompiles every source (objects go to paper_1009_0881_amd/_build).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnmf.so")
PROBES = os.path.join(HERE, "probes")
ARCH = os.environ.get("NMF_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code: the compiler may
# still form them from scalar float code otherwise.
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra) -> str:
    obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON, *extra, "-I", os.path.join(HERE, "..", "include"), "-c", src, "-o", obj]
    if src.endswith(".hip"):
        cmd.insert(1, "-x")
        cmd.insert(2, "hip")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(jobs: int = 8, debug: bool = False, verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    extra = ["-g"] if debug else []
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    probes = build_probes(jobs, extra)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources" + (f" and {len(probes)} probe(s)" if probes else ""))
    return LIB


def build_probes(jobs: int = 8, extra=()) -> list:
    """Standalone measurement programs (probes/*.hip -> probes/<name>), not part of the library."""
    srcs = sorted(glob.glob(os.path.join(PROBES, "*.hip")))

    def one(src):
        exe = os.path.splitext(src)[0]
        cmd = [hipcc(), "-x", "hip", *COMMON, *extra, src, "-o", exe]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
        return exe

    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        return list(ex.map(one, srcs))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args(argv)
    build(a.jobs, a.debug, verbose=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
