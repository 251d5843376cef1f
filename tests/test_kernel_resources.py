"""Register budget of the HIP kernels, from the compiler's resource remarks
recorded when the library is built: no kernel spills to scratch memory (a
spill in a step kernel costs more HBM traffic than the stencil itself)."""
import json
import os

import pytest

from paper_2110_03345_amd import build_lib


def _resources():
    if not os.path.exists(build_lib.RESOURCES):
        pytest.skip("library not built here (no resource remarks)")
    with open(build_lib.RESOURCES) as f:
        return json.load(f)


def test_no_kernel_spills_registers():
    res = _resources()
    steps = [k for k in res if "step2d_" in k or "step3d_" in k]
    assert len(steps) >= 40, len(steps)
    spills = {k: v["scratch"] for k, v in res.items() if v.get("scratch", 0) > 0}
    assert not spills, spills


def test_single_shot_3d_steps_meet_their_occupancy_target():
    """The leapfrog 3D kernels that ask for 4 waves per SIMD (radius-2 or
    narrower row blocks, and the 8-wave forward) stay within 128 VGPRs: the
    target is a compiler attribute, and this checks that it held."""
    import re
    res = _resources()
    seen = 0
    for name, r in res.items():
        m = re.search(r"step3d_kernelILi(\d)ELb(\d)ELi(\d)ELi(\d)ELi(\d)E", name)
        if not m:
            continue
        R, adj, ry, waves, mode = (int(x) for x in m.groups())
        if mode == 0 and (ry <= 2 or (not adj and waves == 8)):
            seen += 1
            assert r["vgpr"] <= 128, (name, r)
    assert seen >= 4, seen
