"""Device-assembly check for the wide-store data hazard (host only).

A buffer store of more than 64 bits reads its data registers after issue; a
VALU instruction that rewrites one of them within the next two instruction
slots can change the stored value.  The compiler inserts the wait states
only when the store's scalar offset is an immediate, so a kernel that passes
a register scalar offset to such a store can store a value it never
computed (seen as the lo word of the first voxel of a 128-bit store
replaced by the next store's out-of-range offset, 0x80000000 = -0.0).
This test compiles every kernel source to gfx950 assembly and fails on any
such pair."""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess

import pytest

from paper_1907_05709_amd import build as B

WINDOW = 2  # wait states a gfx950 wide store needs before its data is rewritten

_STORE = re.compile(
    r"^buffer_store_dwordx([34])\s+v\[(\d+):(\d+)\],\s*\S+,\s*s\[\d+:\d+\],\s*(\S+)")
_VDST = re.compile(r"^(v_\S+)\s+(?:v\[(\d+):(\d+)\]|v(\d+))\b")


def _instructions(asm: str) -> list[str]:
    out = []
    for line in asm.splitlines():
        t = line.split(";")[0].strip()
        if not t or t.startswith(".") or t.endswith(":"):
            continue
        out.append(t)
    return out


def _vdst(ins: str) -> set[int]:
    m = _VDST.match(ins)
    if not m or m.group(1).startswith(("v_cmp_", "v_cmpx_", "v_readfirstlane", "v_readlane")):
        return set()
    if m.group(2):
        return set(range(int(m.group(2)), int(m.group(3)) + 1))
    return {int(m.group(4))}


def store_hazards(asm: str) -> list[str]:
    """Pairs (wide buffer store with register soffset, VALU rewriting its
    data within WINDOW slots)."""
    ins = _instructions(asm)
    found = []
    for i, t in enumerate(ins):
        m = _STORE.match(t)
        if not m or not m.group(4).startswith("s"):
            continue
        data = set(range(int(m.group(2)), int(m.group(3)) + 1))
        slots = 0
        for nxt in ins[i + 1:]:
            if slots >= WINDOW:
                break
            if nxt.startswith("s_nop"):
                parts = nxt.split()
                slots += 1 + (int(parts[1], 0) if len(parts) > 1 else 0)
                continue
            if _vdst(nxt) & data:
                found.append(f"{t}  ->  {nxt}")
                break
            slots += 1
    return found


def _asm(src: str) -> str:
    cmd = [B.HIPCC, *B.CFLAGS, "--cuda-device-only", "-S", "-o", "-",
           os.path.join(B.CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(f"hipcc failed for {src}: {r.stderr[-2000:]}")
    return r.stdout


def test_scanner_flags_the_pattern_and_its_fixes():
    bad = ("buffer_store_dwordx4 v[2:5], v153, s[76:79], s91 offen sc1\n"
           "v_cndmask_b32_e64 v2, v152, v154, s[6:7]\n")
    assert len(store_hazards(bad)) == 1
    imm = bad.replace("s91 offen", "0 offen")
    assert store_hazards(imm) == []
    padded = bad.replace("sc1\n", "sc1\ns_nop 1\n")
    assert store_hazards(padded) == []
    narrow = bad.replace("dwordx4 v[2:5]", "dwordx2 v[2:3]")
    assert store_hazards(narrow) == []


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_kernels_have_no_wide_store_data_hazard():
    with cf.ThreadPoolExecutor(max_workers=min(8, len(B.SOURCES))) as ex:
        asms = dict(zip(B.SOURCES, ex.map(_asm, B.SOURCES)))
    bad = {src: store_hazards(a) for src, a in asms.items()}
    bad = {k: v for k, v in bad.items() if v}
    assert not bad, "\n".join(f"{k}: {v[:3]}" for k, v in bad.items())
    assert any("buffer_store_dwordx4" in a for a in asms.values())
