"""Instruction mix of the direct sum's inner loop, counted in the gfx950 assembly of this build.

Compiles csrc/direct.hip to device assembly with the library's flags, finds the kernel
k_direct<K1, K2, T, LT, no dump, cell centres>, takes its lens loop (the basic block that holds
the reciprocals: the float32 runs between two FP64 additions for the lane's K1 K2 rays) and
counts its instructions by class, per ray-lens interaction.  With the issue rates of rs_probe_issue_rate
this gives the loop's instruction-mix ceiling.

    python -m paper_0905_2453_amd.isa_mix [--block 1x4] [--out profiles/k_direct_isa_mix.json]
"""
from __future__ import annotations

import argparse
import collections
import functools
import hashlib
import json
import os
import re
import subprocess
import tempfile

from . import build as B

CLASSES = {
    "vop2_f32": re.compile(r"^v_(mul|fmac|sub|add|subrev|mac|max|min)_f32_e32$"),
    "vop3_f32": re.compile(r"^v_(fma|mul|sub|add|fmac)_f32(_e64)?$"),
    "rcp_f32": re.compile(r"^v_rcp_f32"),
    "cvt_f64": re.compile(r"^v_cvt_f64_f32"),
    "add_f64": re.compile(r"^v_add_f64"),
    "lds": re.compile(r"^ds_"),
    "s_nop": re.compile(r"^s_nop$"),
}


@functools.lru_cache(maxsize=4)
def _asm(path: str) -> str:
    out = os.path.join(tempfile.mkdtemp(), "direct.s")
    flags = [f for f in B.FLAGS if f != "-fPIC"]
    subprocess.check_call([B.HIPCC, *flags, "--cuda-device-only", "-S", path, "-o", out],
                          stderr=subprocess.DEVNULL)
    return open(out).read()


def count(block=(1, 4), T=0, LT=256) -> dict:
    T = T or (8 if block[0] == 1 else 16)
    src = os.path.join(B.CSRC, "direct.hip")
    lines = _asm(src).split("\n")
    sym = f"k_directILi{block[0]}ELi{block[1]}ELi{T}ELi{LT}ELb0ELb0E"
    start = next(i for i, l in enumerate(lines) if re.match(rf"^_Z.*{sym}.*:", l))
    blocks, cur = collections.OrderedDict(), None
    for l in lines[start + 1:]:
        if "s_endpgm" in l:
            break
        m = re.match(r"^(\.LBB\d+_\d+):", l)
        if m:
            cur = m.group(1)
            blocks[cur] = []
            continue
        t = l.strip()
        if cur and t and not t.startswith((";", ".")):
            blocks[cur].append(t.split()[0])
    # the lens loop: the block with the most reciprocals; one reciprocal serves four rays in
    # one-column blocks, two in several-column ones
    name, ins = max(blocks.items(), key=lambda kv: sum(1 for x in kv[1] if x.startswith("v_rcp_f32")))
    inter = sum(1 for x in ins if x.startswith("v_rcp_f32")) * (4 if block[0] == 1 else 2)
    hist = collections.Counter(ins)
    per = {k: sum(v for op, v in hist.items() if rx.match(op)) / inter for k, rx in CLASSES.items()}
    per["valu_total"] = sum(v for op, v in hist.items() if op.startswith("v_")) / inter
    return {"kernel": f"k_direct<{block[0]},{block[1]},{T},{LT}> (cell centres, no dump)", "block": f"{block[0]}x{block[1]}",
            "fp32_run": T, "lens_tile": LT, "loop_block": name, "interactions_per_loop": inter,
            "per_interaction": per, "loop_histogram": dict(hist.most_common()),
            "source": os.path.relpath(src, B.ROOT), "source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
            "command": "python -m paper_0905_2453_amd.isa_mix --block " + f"{block[0]}x{block[1]}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--block", default="1x4")
    ap.add_argument("--out", default=os.path.join(B.ROOT, "profiles", "k_direct_isa_mix.json"))
    a = ap.parse_args()
    k1, k2 = (int(v) for v in a.block.lower().split("x"))
    res = count((k1, k2))
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")
    print(json.dumps(res["per_interaction"]))


if __name__ == "__main__":
    main()
