"""The hardware property the MFMA shading sums rely on: every K step of
v_mfma_f32_4x4x1f32 and v_mfma_f32_16x16x4f32 rounds as one fused
multiply-add, in K order, under the lane layout the shading code assumes, so
an MFMA chain gives the bits of the fmaf chain over the same products
(paper_2104_00359_amd/csrc/mfma_probe.hip, built by build.py beside the
library).  The probe also prints the FP32 MFMA and VALU rates, which are
recorded but not asserted."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

PROBE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2104_00359_amd", "mfma_probe")


def test_mfma_chains_round_like_fmaf_chains():
    assert os.path.exists(PROBE), "mfma_probe is not built: run __graft_entry__.build()"
    print("running", PROBE, flush=True)
    out = subprocess.run([PROBE], capture_output=True, text=True, timeout=120)
    print(out.stdout, out.stderr, flush=True)
    assert out.returncode == 0, out.stdout + out.stderr
    vals = dict(line.split(None, 1) for line in out.stdout.splitlines() if line.strip())
    assert vals["mfma_4x4x1_bitwise_equal_to_fmaf"].startswith("256 of 256")
    assert vals["mfma_16x16x4_bitwise_equal_to_fmaf"].startswith("256 of 256")
