"""Compile-time resources of the HIP kernels (hipcc's resource-usage
remarks for gfx950): no kernel spills to or indexes into scratch memory,
and the decoders' LDS allows the workgroups per CU their designs count on
(two of the lane decoder, three of the split decoder, 160 KB per CU)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_17849_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def usage():
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    from paper_2602_17849_amd import build as qbuild   # the library's own flags
    cmd = [HIPCC] + [f for f in qbuild.HIPCC_FLAGS if f != "-fPIC"] + [
           "--cuda-device-only", "-c",
           os.path.join(CSRC, "qlc_kernels.hip"), "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+)", line)
        if cur and m:
            kernels[cur][m.group(1).strip()] = int(m.group(2))
    assert kernels
    return kernels


def test_no_scratch(usage):
    for name, u in usage.items():
        assert u.get("ScratchSize", 0) == 0, name
        assert u.get("VGPRs Spill", 0) == 0, name


def test_decoder_lds_budgets(usage):
    lds = {n: u.get("LDS Size", 0) for n, u in usage.items()}
    split = [v for n, v in lds.items() if "k_decode_split" in n]
    lane = [v for n, v in lds.items() if re.search(r"k_decodeILi", n)]
    assert split and lane
    assert all(3 * v <= 160 * 1024 for v in split)
    assert all(2 * v <= 160 * 1024 for v in lane)
