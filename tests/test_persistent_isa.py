"""The persistent batch kernel's loop structure in its compiled gfx950 code (CPU only:
hipcc cross-compiles).

The kernel's task loop must be one loop whose exit is a scalar (wave-uniform) branch, with
no inner loop that contains a workgroup barrier.  The first version of the kernel kept its
task number in LDS and took the next ticket in lane 0 next to the loop's back edge: the
structurizer nested a lane-divergent inner loop around the barrier and the task, in which
lanes 1..63 of wave 0 re-ran the last task while lane 0, which writes the next task, waited
outside it, so the launch never ended.  All lane-0 work is now in a called function
(next_task) and the task number is read with readfirstlane.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def kernel_asm(tmp_path, name):
    src = os.path.join(ROOT, "paper_1612_05778_amd", "csrc", "persistent.hip")
    out = tmp_path / "persistent.s"
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form=true", "-I",
           os.path.join(ROOT, "include"), "-I",
           os.path.join(ROOT, "paper_1612_05778_amd", "csrc"), "-x", "hip", "--cuda-device-only",
           "-S", src, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    text = out.read_text().splitlines()
    start = next(i for i, ln in enumerate(text) if re.match(rf"^_ZN3zpm\d+{name}\w*:", ln))
    end = next(i for i in range(start, len(text)) if text[i].startswith(".Lfunc_end"))
    return text[start:end]


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="no hipcc")
def test_task_loop_has_no_divergent_inner_loop(tmp_path):
    asm = kernel_asm(tmp_path, "k_batch_persistent")
    depth = 0
    barriers = []
    for ln in asm:
        m = re.search(r"Depth=(\d+)", ln)
        if ln.startswith(".LBB") or ln.startswith("; %bb"):
            depth = int(m.group(1)) if m else 0
        if "s_barrier" in ln:
            barriers.append(depth)
    assert barriers, "the task loop has no barrier"
    assert all(d <= 1 for d in barriers), f"a barrier sits in a nested loop (depths {barriers})"
    assert not any("Depth=2" in ln for ln in asm), "the task loop has an inner loop"
    # the loop is left on a condition computed from readfirstlane (scalar registers)
    cond = [i for i, ln in enumerate(asm) if re.search(r"v_cmp_\w+_e64 s\[\d+:\d+\], s\[", ln)]
    assert cond, "no scalar loop-exit comparison"
    calls = [ln for ln in asm if "s_swappc_b64" in ln]
    assert len(calls) >= 2    # next_task, then the task
