"""Structural check of the compiled gfx950 kernels: no loop that holds a barrier may be
controlled per lane.

The AMDGPU backend lowers a loop whose exit differs between lanes by masking
the exited lanes out of `exec` and branching on `exec` (`s_andn2_b64 exec, exec,
...` followed by `s_cbranch_execz`/`s_cbranch_execnz`).  If such a loop holds an
`s_barrier`, the lanes still inside keep meeting the barrier while the exited
lanes wait outside the loop, and the workgroup can hang.  Every loop with a
barrier must therefore be controlled by scalar (SCC/VCC) branches.
"""
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

LABEL = re.compile(r"^(\.LBB\d+_\d+):")
FUNC = re.compile(r"^([A-Za-z_][\w.$]*):\s*(;.*)?$")


def device_asm(src_path, out_path):
    from paper_2504_08081_amd import _build
    cmd = [_build.hipcc()] + _build.HIP_FLAGS + ["-I", _build.INCLUDE, "-I", _build.CSRC, "-x", "hip",
                                                  "--cuda-device-only", "-S", "-o", out_path, src_path]
    subprocess.run(cmd, check=True, stderr=subprocess.DEVNULL)
    return open(out_path).read()


def per_lane_loops_with_barrier(asm_text):
    """[(function, header label)] of loops holding a barrier whose control is per lane."""
    lines = asm_text.splitlines()
    bad = []
    func = None
    label_pos = {}
    for i, ln in enumerate(lines):
        m = FUNC.match(ln)
        if m and not ln.startswith(".") and not ln.startswith("\t"):
            func = m.group(1)
        m = LABEL.match(ln)
        if m:
            label_pos[(func, m.group(1))] = i
    func = None
    for i, ln in enumerate(lines):
        m = FUNC.match(ln)
        if m and not ln.startswith(".") and not ln.startswith("\t"):
            func = m.group(1)
        s = ln.strip()
        if not re.match(r"s_andn2_b64\s+exec,\s*exec,", s):
            continue
        nxt = lines[i + 1].strip() if i + 1 < len(lines) else ""
        mb = re.match(r"s_cbranch_exec(n?z)\s+(\.LBB\d+_\d+)", nxt)
        if not mb:
            continue
        kind, target = mb.group(1), mb.group(2)
        tpos = label_pos.get((func, target))
        if tpos is None:
            continue
        if kind == "nz" and tpos <= i:
            region = lines[tpos:i + 1]
            header = target
        elif kind == "z" and tpos > i:
            # exit branch; the loop header is the label that follows, its body runs to the exit
            j = i + 2
            while j < len(lines) and not LABEL.match(lines[j]):
                j += 1
            if j >= len(lines) or not any("Loop Header" in x for x in lines[j:j + 3]):
                continue
            header = LABEL.match(lines[j]).group(1)
            region = lines[j:tpos]
        else:
            continue
        if any(r.strip().startswith("s_barrier") for r in region):
            bad.append((func, header))
    return bad
