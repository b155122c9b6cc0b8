"""Code-generation guards for the temporally blocked passes (no GPU needed).

The tile pass keeps a batch of region loads in flight per thread (one per
load unit of its wave) before it bit-packs any of them.  If the compiler moves work that uses a loaded value
into the load's own conditional block, it has to wait for that load there
(`s_waitcnt vmcnt(0)` right after it) and the batch is serialised, which cost
8 % of the pass at rho = 256 when it happened.  These tests compile the passes
to gfx950 assembly and check that no life region load is waited on inside its
block, and that the diffusion pass issues all its region loads before its
first wait on them (it clears its LDS planes meanwhile).
"""
import os
import re
import subprocess

import pytest

from paper_1706_04552_amd import build as B

SRC = os.path.join(B.CSRC, "sg_life_tb.hip")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(B.HIPCC):
        pytest.skip("hipcc is not available")
    out = tmp_path_factory.mktemp("asm") / "sg_life_tb.s"
    cmd = [B.HIPCC, *B.HIP_FLAGS, "--cuda-device-only", "-S", SRC, "-o", str(out)]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out.read_text()


def _kernels(text):
    names = re.findall(r"^(_Z\w*k_life_tb\w*):", text, re.M)
    for name in names:
        start = text.index(name + ":")
        end = text.index(".Lfunc_end", start)
        lines = [l.strip() for l in text[start:end].split("\n")]
        yield name, [l for l in lines if l and not l.startswith(";")]


def _waited_at_once(lines):
    """Region loads (16-byte) followed by a full vmcnt wait before their block ends."""
    bad = 0
    for i, line in enumerate(lines):
        if not re.match(r"(global|flat)_load_dwordx4\b", line):
            continue
        for nxt in lines[i + 1:i + 8]:
            if nxt.startswith(".LBB") or nxt.startswith("s_cbranch") or nxt.startswith("s_or_b64 exec"):
                break
            if "vmcnt(0)" in nxt:
                bad += 1
                break
    return bad


def _bit_loads_per_thread(name):
    """Region loads per thread of a pass that reads bit-packed tiles (None
    for a pass reading bytes): 4-row units of the region's word columns
    (the tile's, one each side) over its rows at 32 generations, spread over
    the workgroup's threads."""
    m = re.search(r"k_life_tb_bitsILi(\d+)ELb[01]ELb1ELb[01]ELi(\d+)E", name)
    c = re.search(r"k_life_tb_compact_bitsILi(\d+)ELb1ELb[01]E", name)
    if m:
        rho, threads = int(m.group(1)), int(m.group(2))
    elif c:
        rho, threads = int(c.group(1)), 256
    else:
        return None
    units = (rho // 32 + 2) * (rho // 4 + 2 * 8)
    return -(-units // threads)


def test_tile_pass_region_loads_stay_in_flight(asm):
    kernels = list(_kernels(asm))
    # dense (both maps, four sides; rho = 256 at two workgroup sizes),
    # compact, batch, and the passes to and from bit-packed tiles (both maps,
    # four sides, three directions; rho = 256 at two workgroup sizes; and
    # the compact ones, three sides, three directions)
    assert len(kernels) >= 10 + 30 + 9
    for name, lines in kernels:
        loads = sum(1 for l in lines if re.match(r"(global|flat)_load_dwordx4\b", l))
        per_thread = _bit_loads_per_thread(name)
        # a wave's batch of region loads (one per load unit)
        assert loads >= (2 if per_thread is None else per_thread), name
        assert _waited_at_once(lines) == 0, name


def test_guard_detects_a_serialised_batch():
    # the pattern the guard exists for: a load whose block waits for it at once
    lines = ["s_cbranch_execz .LBB0_2", "v_lshl_add_u64 v[2:3], v[4:5], 0, v[2:3]",
             "global_load_dwordx4 v[6:9], v[2:3], off", "s_waitcnt vmcnt(0)",
             "v_lshlrev_b32_e32 v10, 1, v7", ".LBB0_2:"]
    assert _waited_at_once(lines) == 1
    ok = ["global_load_dwordx4 v[6:9], v[2:3], off", ".LBB0_2:", "s_waitcnt vmcnt(0)"]
    assert _waited_at_once(ok) == 0


@pytest.fixture(scope="module")
def diffuse_asm(tmp_path_factory):
    if not os.path.exists(B.HIPCC):
        pytest.skip("hipcc is not available")
    out = tmp_path_factory.mktemp("asm") / "sg_diffuse_tb.s"
    src = os.path.join(B.CSRC, "sg_diffuse_tb.hip")
    cmd = [B.HIPCC, *B.HIP_FLAGS, "--cuda-device-only", "-S", src, "-o", str(out)]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out.read_text()


def test_diffusion_tile_pass_issues_all_region_loads_before_waiting(diffuse_asm):
    # the diffusion pass lists its chunks while every region load is in flight
    names = re.findall(r"^(_Z\w*k_diffuse_tb\w*):", diffuse_asm, re.M)
    assert len(names) == 12  # rho 16, 32, 64 for both maps, halo 8 and 16
    for name in names:
        start = diffuse_asm.index(name + ":")
        end = diffuse_asm.index(".Lfunc_end", start)
        lines = [l.strip() for l in diffuse_asm[start:end].split("\n")]
        lines = [l for l in lines if l and not l.startswith(";")]
        loads = [i for i, l in enumerate(lines) if re.match(r"global_load_dwordx4\b", l)]
        assert loads, name
        assert not [l for l in lines[loads[0]:loads[-1]] if "vmcnt" in l], name
