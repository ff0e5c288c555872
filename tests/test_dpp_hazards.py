"""Listing check of the DPP reads in the compiled update kernels (host only).

A DPP read of a VGPR needs two wait states after a VALU instruction wrote
it. The compiler inserts them for its own DPP moves, but not for the DPP
source of an FMA written as inline asm (the 64x64 Cholesky factor). This
test compiles update.hip to gfx950 assembly and checks every DPP
instruction: no VALU write of its DPP source within the two preceding wait
states (s_nop N counts N + 1, any other instruction one). The scanner is
itself checked on a planted listing."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2509_26222_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_26222_amd", "csrc")


def _vregs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]$", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def dpp_hazards(listing):
    """(number of DPP instructions, list of (writer, dpp reader) pairs)."""
    ins = []
    for line in listing.splitlines():
        t = line.strip()
        if not t or t.startswith(";") or t.startswith(".") or t.endswith(":"):
            continue
        ins.append(t)
    found, n = [], 0
    for i, t in enumerate(ins):
        op = t.split()[0]
        if "_dpp" not in op:
            continue
        n += 1
        ops = t.split(None, 1)[1].split(",")
        src = _vregs(ops[1].strip().split()[0].lstrip("-"))
        waits, j = 0, i - 1
        while j >= 0 and waits < 2:
            p = ins[j]
            pop = p.split()[0]
            if pop.startswith("s_nop"):
                waits += int(p.split()[1]) + 1
            else:
                if pop.startswith("v_") and len(p.split()) > 1:
                    dst = _vregs(p.split(None, 1)[1].split(",")[0].strip())
                    if dst & src:
                        found.append((p, t))
                        break
                waits += 1
            j -= 1
    return n, found


def test_scanner_finds_planted_hazards():
    planted = "\n".join([
        "\tv_mov_b32_e32 v2, v5",
        "\tv_fmac_f64_dpp v[6:7], v[2:3], v[8:9] row_newbcast:1 row_mask:0xf bank_mask:0xf",
        "\tv_add_f64 v[10:11], v[0:1], v[0:1]",
        "\ts_nop 1",
        "\tv_mov_b32_dpp v12, v10 row_newbcast:2 row_mask:0xf bank_mask:0xf",
        "\tv_add_f64 v[14:15], v[0:1], v[0:1]",
        "\ts_nop 0",
        "\tv_mov_b32_dpp v12, v14 row_newbcast:2 row_mask:0xf bank_mask:0xf",
    ])
    n, found = dpp_hazards(planted)
    assert n == 3
    assert [f[1].split()[0] for f in found] == ["v_fmac_f64_dpp", "v_mov_b32_dpp"]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_update_kernels_have_no_dpp_source_hazard():
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "update.s")
        # the library's own compile flags, device code only, as assembly
        cmd = [build.HIPCC, *build.COMMON, "--cuda-device-only", "-S",
               os.path.join(CSRC, "update.hip"), "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        listing = open(out).read()
    n, found = dpp_hazards(listing)
    assert n > 500  # the factor's fused updates are there
    assert "v_fmac_f64_dpp" in listing
    assert not found, found[:5]
