"""Build libpst.so (the HIP library) in-tree for gfx950.

    python -m paper_1206_3215_amd.build [--force] [-j N]

Every csrc/*.hip and csrc/*.cpp is compiled by hipcc to _build/*.o (in
parallel) and linked into paper_1206_3215_amd/libpst.so.  Without --force,
objects newer than their source and every header are reused.  Rebuilt
device code is then checked by store_audit (a gfx950 store hazard).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libpst.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC, "-I", os.path.join(ROOT, "include"),
    "-Wno-unused-command-line-argument",
]


def _sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _headers():
    return glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h"))


def _compile(src: str, obj: str) -> tuple[str, int, str]:
    cmd = [HIPCC, *COMMON, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 target feature; drop that noise
    err = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in line and "unknown target feature" not in line)
    return src, r.returncode, err


def build(force: bool = False, jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    hdr_t = max((os.path.getmtime(h) for h in _headers()), default=0.0)
    todo = []
    objs = []
    for s in srcs:
        o = os.path.join(BUILD, os.path.basename(s) + ".o")
        objs.append(o)
        if force or not os.path.exists(o) or os.path.getmtime(o) < max(os.path.getmtime(s), hdr_t):
            todo.append((s, o))
    jobs = jobs or min(8, os.cpu_count() or 1)
    failed = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, rc, err in ex.map(lambda so: _compile(*so), todo):
            if verbose:
                print(f"[build] {'ok ' if rc == 0 else 'ERR'} {os.path.relpath(src, ROOT)}", flush=True)
            if rc != 0:
                failed.append((src, err))
    if failed:
        for src, err in failed:
            print(f"--- {src}\n{err}", file=sys.stderr)
        raise RuntimeError(f"hipcc failed for {len(failed)} source(s)")
    if todo or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
        os.replace(tmp, LIB)
        if verbose:
            print(f"[build] linked {os.path.relpath(LIB, ROOT)}", flush=True)
    if todo:
        # every rebuilt device object must be free of the wide-store hazard
        from paper_1206_3215_amd import store_audit
        bad = store_audit.audit([o for s, o in todo if s.endswith(".hip")])
        if bad:
            for b in bad[:20]:
                print(" | ".join(str(x) for x in b), file=sys.stderr)
            os.remove(LIB)
            raise RuntimeError(f"{len(bad)} wide store(s) whose data registers are overwritten too early "
                               "(see paper_1206_3215_amd/store_audit.py)")
        if verbose:
            print("[build] store audit clean", flush=True)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    build(force=a.force, jobs=a.j)
