"""Check of the built device code for one gfx950 hazard.

A vector memory store of more than 8 bytes reads its data registers over
more than one cycle; on gfx950 an instruction that overwrites those
registers right behind the store can make it write the new values (seen as
run-to-run differences in FP64 results, with no wait state between the
two in the compiler's output).  The kernels therefore issue 16-byte stores
from an asm statement that ends with two wait states, and store everything
else 8 bytes at a time.  This module disassembles the gfx950 code objects of
the built objects (this project's own code) and reports every wide store
followed by a write of one of its data registers within two wait states.

    python -m paper_1206_3215_amd.store_audit [objects...]
"""
from __future__ import annotations

import glob
import os
import re
import subprocess
import sys
import tempfile

LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"
MIN_WAIT_STATES = 2

_WIDE = re.compile(r"^(buffer|global|flat|scratch)_store_(dwordx[34]|b96|b128)\b")
_REG = re.compile(r"^v\[(\d+):(\d+)\]$|^v(\d+)$")
_FN = re.compile(r"^([0-9a-f]+) <(\S+)>:")


def _vregs(tok: str) -> set:
    m = _REG.match(tok.strip())
    if not m:
        return set()
    if m.group(1):
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    return {int(m.group(3))}


def _writes(mn: str, ops: list) -> set:
    """VGPRs an instruction writes (its first operand, for the kinds that
    have a vector destination)."""
    if not ops:
        return set()
    if mn.startswith("v_") and not mn.startswith(("v_cmp", "v_readlane", "v_readfirstlane")):
        return _vregs(ops[0])
    if mn.startswith(("ds_read", "ds_load", "buffer_load", "global_load", "flat_load", "scratch_load")):
        return _vregs(ops[0])
    return set()


def _wait_states(mn: str, ops: list) -> int:
    if mn == "s_nop":
        return int(ops[0], 0) + 1 if ops else 1
    return 1


def audit_disassembly(lines) -> list:
    """[(function, store, offending instruction, wait states between)]"""
    bad = []
    fn = "?"
    pending = []  # [regs, store text, wait states so far]
    for raw in lines:
        line = raw.split("//")[0].strip()
        m = _FN.match(line)
        if m:
            fn, pending = m.group(2), []
            continue
        if not line or line.endswith(":"):
            continue
        parts = line.split(None, 1)
        mn = parts[0]
        ops = [o.strip() for o in parts[1].split(",")] if len(parts) > 1 else []
        w = _writes(mn, ops)
        keep = []
        for regs, text, ws in pending:
            if w & regs:
                bad.append((fn, text, line, ws))
                continue
            ws += _wait_states(mn, ops)
            if ws < MIN_WAIT_STATES:
                keep.append([regs, text, ws])
        pending = keep
        if _WIDE.match(mn) and ops:
            data = ops[1] if mn.startswith(("global", "flat", "scratch")) else ops[0]
            pending.append([_vregs(data), line, 0])
        if mn in ("s_endpgm", "s_branch", "s_setpc_b64") or mn.startswith("s_cbranch"):
            # the hazard does not follow a branch in this scan; a taken
            # branch's target starts with the wait states of the branch
            pending = [p for p in pending if p[2] + 1 < MIN_WAIT_STATES]
    return bad


def audit_object(obj: str) -> list:
    with tempfile.TemporaryDirectory() as tmp:
        fat = os.path.join(tmp, "fat.bin")
        co = os.path.join(tmp, "dev.co")
        subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", obj, fat], check=True)
        if os.path.getsize(fat) == 0:
            return []
        subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--targets={TARGET}",
                        f"--input={fat}", f"--output={co}"], check=True)
        dis = subprocess.run([f"{LLVM}/llvm-objdump", "-d", "--mcpu=gfx950", co], check=True,
                             capture_output=True, text=True).stdout
    return audit_disassembly(dis.splitlines())


def audit(objs) -> list:
    bad = []
    for o in objs:
        bad += [(os.path.basename(o),) + b for b in audit_object(o)]
    return bad


if __name__ == "__main__":
    from paper_1206_3215_amd import build as _b
    objs = sys.argv[1:] or sorted(glob.glob(os.path.join(_b.BUILD, "*.hip.o")))
    bad = audit(objs)
    for b in bad[:20]:
        print(*b, sep=" | ")
    print(f"{len(bad)} wide store(s) with a data register overwritten within {MIN_WAIT_STATES} wait states")
    sys.exit(1 if bad else 0)
