"""Build libgscl.so (HIP, gfx950) in-tree.

Every ``csrc/*.hip`` file is one compile unit; units compile in parallel and
link into ``paper_1207_1746_amd/libgscl.so``.  ``force=False`` rebuilds only
objects older than their source or any header.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgscl.so")

ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # no packed-FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def _compile(src: str, obj: str) -> tuple[str, int, str]:
    cmd = [_hipcc(), *FLAGS, "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    return src, p.returncode, p.stdout + p.stderr


def build(force: bool = True, jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    headers = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    newest_hdr = max((os.path.getmtime(h) for h in headers), default=0.0)
    todo, objs = [], []
    for s in sources:
        o = os.path.join(BUILD, os.path.basename(s)[:-4] + ".o")
        objs.append(o)
        if force or not os.path.exists(o) or os.path.getmtime(o) < max(os.path.getmtime(s), newest_hdr):
            todo.append((s, o))
    jobs = jobs or min(len(todo) or 1, os.cpu_count() or 4, 16)
    failed = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, rc, out in ex.map(lambda so: _compile(*so), todo):
            if verbose or rc:
                sys.stderr.write(f"[build] {os.path.basename(src)} rc={rc}\n{out}")
            if rc:
                failed.append(src)
    if failed:
        raise RuntimeError("HIP compile failed: " + ", ".join(os.path.basename(f) for f in failed))
    if todo or force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        p = subprocess.run([_hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs],
                           capture_output=True, text=True)
        if p.returncode:
            raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import time
    t = time.time()
    build(force="--force" in sys.argv, verbose="-v" in sys.argv)
    print(f"built {LIB} in {time.time() - t:.1f}s")
