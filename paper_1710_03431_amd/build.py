"""Builds libaqt.so in-tree with hipcc for gfx950.

    python -m paper_1710_03431_amd.build      (or build() from Python)

Each HIP source is compiled to an object of its own (in parallel, under _build/ at the
repository root), then the objects are linked into the shared library.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaqt.so")
OBJ_DIR = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wno-unused-result",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _run(cmd, env):
    res = subprocess.run(cmd, capture_output=True, text=True, env=env)
    if res.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res.returncode


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    env = dict(os.environ)
    env.setdefault("TMPDIR", "/tmp")
    os.makedirs(OBJ_DIR, exist_ok=True)
    incs = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-DAQT_BUILD"]
    objs, cmds = [], []
    for src in sources():
        obj = os.path.join(OBJ_DIR, os.path.basename(src)[:-4] + ".o")
        objs.append(obj)
        cmds.append([hipcc, *HIPCC_FLAGS, *incs, "-c", src, "-o", obj])
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    workers = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        codes = list(ex.map(lambda c: _run(c, env), cmds))
    if any(codes):
        raise RuntimeError("hipcc failed compiling libaqt sources")
    tmp = LIB + ".tmp"
    link = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    if _run(link, env):
        raise RuntimeError("hipcc failed linking libaqt.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
