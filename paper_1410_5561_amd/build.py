"""Build the gfx950 stencil library (libmwdstencil.so) in-tree with hipcc.

    python -m paper_1410_5561_amd.build [--force] [--jobs N] [--resource-usage]

Every translation unit under csrc/ is compiled for gfx950 (no other target),
with FP contraction off (the kernels keep the listings' rounding order) and
packed FP32 instructions disabled, then linked into one shared library next
to this file.  Objects go to _build/ at the repository root.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmwdstencil.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


_INCLUDE = re.compile(r'^\s*#\s*include\s+"([^"]+)"', re.M)


def _deps(src, seen=None):
    """The file and every local header it includes, transitively."""
    seen = set() if seen is None else seen
    src = os.path.normpath(src)
    if src in seen or not os.path.exists(src):
        return seen
    seen.add(src)
    with open(src) as f:
        text = f.read()
    for inc in _INCLUDE.findall(text):
        _deps(os.path.join(os.path.dirname(src), inc), seen)
    return seen


def _deps_mtime(src):
    return max(os.path.getmtime(d) for d in _deps(src))


def _obj(src):
    return os.path.join(BUILD, os.path.basename(src) + ".o")


def _compile(src, resource_usage):
    obj = _obj(src)
    cmd = [HIPCC] + CFLAGS + ["-c", src, "-o", obj + ".tmp"]
    if resource_usage:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    p = subprocess.run(cmd, capture_output=True, text=True)
    log = "\n".join(l for l in (p.stdout + p.stderr).splitlines()
                    if "is not a recognized feature for this target" not in l)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, log))
    os.replace(obj + ".tmp", obj)
    return src, log


def build(force: bool = False, jobs: int | None = None, resource_usage: bool = False,
          verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    todo = []
    for s in sources():
        o = _obj(s)
        if force or not os.path.exists(o) or os.path.getmtime(o) < _deps_mtime(s):
            todo.append(s)
    jobs = jobs or min(8, os.cpu_count() or 4)
    logs = {}
    if todo:
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            for src, log in ex.map(lambda s: _compile(s, resource_usage), todo):
                logs[src] = log
                if verbose:
                    print("compiled", os.path.basename(src), flush=True)
    objs = [_obj(s) for s in sources()]
    if todo or not os.path.exists(LIB) or force:
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
        p = subprocess.run(cmd, capture_output=True, text=True)
        if p.returncode != 0:
            raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
        os.replace(tmp, LIB)
    if resource_usage:
        with open(os.path.join(BUILD, "resource_usage.log"), "w") as f:
            for k in sorted(logs):
                f.write("### %s\n%s\n" % (os.path.basename(k), logs[k]))
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--resource-usage", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.force, a.jobs, a.resource_usage, verbose=True))


if __name__ == "__main__":
    sys.exit(main())
