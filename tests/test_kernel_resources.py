"""Register and LDS budgets of the gfx950 kernels, read from the compiler's
resource report (no GPU needed). The heavy tier is sized for 16 waves per
CU (4 per SIMD): if its registers grow past 128 per lane or its LDS past a
quarter of 160 KiB (256-thread workgroups), fewer workgroups fit and the
persistent grid shrinks."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2201_11326_amd import build

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def resource_report(tmp_path):
    src = os.path.join(build.CSRC, "slg_kernels.hip")
    cmd = [HIPCC, *build.flags(), "--offload-device-only", "-c", src, "-o", str(tmp_path / "k.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    assert proc.returncode == 0, proc.stderr[-2000:]
    rows, cur = {}, None
    for line in proc.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            rows[cur] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]|"
                      r"LDS Size \[bytes/block\]): (\d+)", line)
        if m and cur:
            rows[cur][m.group(1).split()[0]] = int(m.group(2))
    return rows


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_kernel_register_lds_budgets(tmp_path):
    rows = resource_report(tmp_path)
    heavy = {k: v for k, v in rows.items() if "heavy_kernel" in k}
    assert len(heavy) == 5, sorted(rows)  # count, emit, wide count, wide emit, count with store
    text = open(os.path.join(build.CSRC, "slg_internal.h")).read()
    threads = int(re.search(r"kHeavyThreads = (\d+);", text).group(1))
    per_cu = 16 // (threads // 64)  # workgroups that make 16 waves per CU
    for name, r in heavy.items():
        assert r["VGPRs"] <= 128 and r["Occupancy"] >= 4, (name, r)
        assert per_cu * r["LDS"] <= 160 * 1024, (name, r, per_cu)
    # the dense tier: 512-thread workgroups, two per CU (8 waves per SIMD
    # would need <= 64 VGPRs; two workgroups need <= 128 and 2 x LDS <= 160 KiB)
    dense = {k: v for k, v in rows.items() if "dense_kernel" in k}
    assert len(dense) == 2, sorted(rows)  # count, emit
    for name, r in dense.items():
        assert r["VGPRs"] <= 128 and r["Occupancy"] >= 4, (name, r)
        assert 2 * r["LDS"] <= 160 * 1024, (name, r)
    for name, r in rows.items():
        assert r.get("ScratchSize", 0) == 0, (name, r)  # no register spills
