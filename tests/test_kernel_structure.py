"""CPU check of the compiled gfx950 kernels (no GPU needed): every loop that holds a
barrier has uniform (scalar) loop control, so no wave can be split around a barrier."""
import os
import re

import pytest

from asm_structure import device_asm, per_lane_loops_with_barrier

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2504_08081_amd", "csrc")


@pytest.mark.parametrize("src", ["sb_bandflux.hip", "sb_fit.hip", "sb_probe.hip"])
def test_no_barrier_in_per_lane_loop(src, tmp_path):
    asm = device_asm(os.path.join(CSRC, src), str(tmp_path / "k.s"))
    if "s_barrier" not in asm:
        # one-wave workgroups: the compiler drops the barriers altogether
        sizes = set(int(v) for v in re.findall(r"\.max_flat_workgroup_size:\s+(\d+)", asm))
        assert sizes and max(sizes) <= 64, sizes
    bad = per_lane_loops_with_barrier(asm)
    assert bad == [], f"loops holding a barrier with per-lane control: {bad}"


def test_checker_flags_a_per_lane_loop_with_barrier():
    """The checker itself: a hand-made loop with exec-controlled exit around a barrier is flagged."""
    asm = "\n".join([
        "k:", ".LBB0_1:", "; =>This Loop Header: Depth=1", "\ts_barrier", "\tv_add_u32 v1, v1, v2",
        "\ts_andn2_b64 exec, exec, s[4:5]", "\ts_cbranch_execnz .LBB0_1", "\ts_endpgm",
    ])
    assert per_lane_loops_with_barrier(asm) == [("k", ".LBB0_1")]
    ok = asm.replace("s_andn2_b64 exec, exec, s[4:5]", "s_cmp_lg_u32 s1, 0").replace(
        "s_cbranch_execnz", "s_cbranch_scc1")
    assert per_lane_loops_with_barrier(ok) == []
