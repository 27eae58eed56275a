"""The build's device code carries no packed FP32 instructions: the gfx950
device pass honours the -packed-fp32-ops target feature in build.FLAGS
(only hipcc's host pass warns that it does not know it).  Checked on the
generated assembly of one kernel file, with and without the feature."""
import os
import re
import subprocess

import pytest

from paper_2509_17083_amd import build as B

PACKED = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")


def _device_asm(flags, src, out):
    cmd = [B.HIPCC, *[f for f in flags if f != "-fPIC"], "--offload-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return open(out).read()


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_device_code_has_no_packed_fp32(tmp_path):
    src = os.path.join(B.CSRC, "ssim.hip")
    with_flag = _device_asm(B.FLAGS, src, str(tmp_path / "with.s"))
    assert len(PACKED.findall(with_flag)) == 0
    i = B.FLAGS.index("-packed-fp32-ops")
    without = B.FLAGS[:i - 3] + B.FLAGS[i + 1:]
    plain = _device_asm(without, src, str(tmp_path / "without.s"))
    # the check can fail: the same file does use them without the feature
    assert len(PACKED.findall(plain)) > 0
