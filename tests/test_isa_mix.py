"""The direct sum's lens-loop instruction mix, counted in this build's gfx950 assembly (no GPU).

The bench prices this mix at the measured issue rates to get the loop's ceiling, so the counts
must say what the kernel does: one reciprocal per four rays in one-column blocks (per two in
several-column ones), one FP64 conversion and addition per ray and component for every group of
float32 runs, and at least the FP32 arithmetic that each interaction needs.  The committed record
must also belong to the committed source.  (One device-assembly compile of direct.hip, shared by
the tests: a few minutes on one core.)
"""
import hashlib
import json
import os
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                                reason="hipcc not available")


def test_one_column_loop_mix():
    from paper_0905_2453_amd import isa_mix
    r = isa_mix.count((1, 4))
    k = r["per_interaction"]
    assert r["fp32_run"] == 8
    assert k["rcp_f32"] == 0.25                     # four rows per reciprocal
    assert k["cvt_f64"] == k["add_f64"] == 1 / 16   # runs of 8, four runs per FP64 addition
    assert k["vop2_f32"] + k["vop3_f32"] >= 7.0      # 28 FP32 operations per lens and four rays
    assert k["vop2_f32"] + k["vop3_f32"] <= 7.5


def test_several_column_loop_mix():
    from paper_0905_2453_amd import isa_mix
    k = isa_mix.count((2, 4))["per_interaction"]
    assert k["rcp_f32"] == 0.5                      # row pairs
    assert k["cvt_f64"] == k["add_f64"] == 1 / 8    # runs of 16, each added in FP64


def test_committed_record_matches_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_direct_isa_mix.json")))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    assert rec["source_sha256"] == hashlib.sha256(src).hexdigest()
    assert rec["block"] == "1x4" and rec["fp32_run"] == 8
