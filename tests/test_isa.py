"""Checks on the gfx950 code the library is built from (CPU: hipcc cross-compiles).

* no packed FP32 instructions (the build disables them; hand-written ones are banned);
* no scratch (private segment) and no register spills in any kernel;
* the filter's inner loop spends one v_exp_f32 per tap.
"""
import os
import re
import shutil

import pytest

from paper_1812_07122_amd import build as b

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                                reason="hipcc not available")

SOURCES = [s for s in b.sources() if s.endswith(".hip")]


@pytest.fixture(scope="module")
def asm():
    return {os.path.basename(s): b.device_asm(s) for s in SOURCES}


def test_no_packed_fp32(asm):
    for name, text in asm.items():
        hits = re.findall(r"\bv_pk_(?:add|mul|fma|mov)_f32\b", text)
        assert not hits, f"{name}: packed FP32 instructions {sorted(set(hits))}"


def test_no_scratch_or_spills(asm):
    for name, text in asm.items():
        for m in re.finditer(r"\.private_segment_fixed_size:\s+(\d+)", text):
            assert int(m.group(1)) == 0, f"{name}: kernel uses scratch"
        for m in re.finditer(r"\.(?:v|s)gpr_spill_count:\s+(\d+)", text):
            assert int(m.group(1)) == 0, f"{name}: register spills"


def test_filter_one_exp_per_tap(asm):
    text = asm["blf_kernel.hip"]
    prefix = "_ZN5blfls16blf_field_kernelILi9ELi8ELi4ELb0ELb0EE"  # direct launch, self-guided, R = 9
    start = text.index(prefix)
    start = text.index(":", start)
    body = text[start:text.index("s_endpgm", start)].split("\n")
    counts = []
    for i, line in enumerate(body):
        if "Loop Header" not in line:
            continue
        label = line.split(":")[0].strip()
        exps = 0
        for later in body[i + 1:]:
            if re.search(r"s_cbranch_\w+\s+" + re.escape(label) + r"\b", later):
                break
            exps += bool(re.match(r"\s*v_exp_f32", later))
        counts.append(exps)
    # the runtime dx loop evaluates K outputs x (2R+1) rows: one exp per tap
    assert 8 * 19 in counts, counts


def _blocks(text, prefix):
    """Instruction lines of every basic block (label to label) of one kernel."""
    start = text.index(prefix)
    start = text.index(":", start)
    body = text[start:text.index("s_endpgm", start)].split("\n")
    blocks, cur = [], []
    for line in body:
        if re.match(r"\s*\.LBB\S+:", line):
            blocks.append(cur)
            cur = []
        elif line.strip() and not line.strip().startswith(";"):
            cur.append(line.strip())
    blocks.append(cur)
    return blocks


def test_pair_filter_one_exp_per_pair(asm):
    """The symmetric-pair kernel evaluates every unordered pair of taps once: at
    R = 24 (blocks of K = 4 rows) each step of its two column-offset loops is one
    straight block of K (R + 1) = 100 or K R = 96 pairs with one exp each and seven
    VALU instructions per pair (difference, exponent FMA, exp, two FMACs and two
    adds, the sums of both pixels)."""
    text = asm["blf_pair_kernel.hip"]
    counts = []
    for lines in _blocks(text, "_ZN5blfls15blf_pair_kernelILi24ELb0ELb0EE"):
        exps = sum(bool(re.match(r"v_exp_f32", l)) for l in lines)
        if exps:
            valu = sum(bool(re.match(r"v_", l)) for l in lines)
            counts.append(exps)
            assert valu <= 7.05 * exps, (exps, valu)
    assert sorted(counts) == [96, 100], counts
