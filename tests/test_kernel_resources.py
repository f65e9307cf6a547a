"""The hot kernels keep their per-thread state in registers: compiled for
gfx950, no kernel of the certificate, merge, batched and bridge-step sources
uses private (scratch) memory.  A spilled register or an array the compiler
could not keep in registers would put every thread's working set in memory
beside the union-find state (one extra call site of the edge stream in the
one-workgroup-per-node kernel once did this: 256 bytes per lane, the large
query 161 -> 191 ms)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_07346_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOT = ["solo_kernels.hip", "cert_kernels.hip", "batched_kernels.hip", "bridge_kernels.hip"]


def resources(src, tmp_path):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src), "-o",
           str(tmp_path / (src + ".o")), "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"remark:\s+ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            out[name] = int(m.group(1))
    return out


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
@pytest.mark.parametrize("src", HOT)
def test_hot_kernels_use_no_scratch(src, tmp_path):
    res = resources(src, tmp_path)
    assert res, "no kernel resource report for %s" % src
    assert {k: v for k, v in res.items() if v != 0} == {}
