"""The XCD-aware launch maps of the outer passes (map_block / xcd_slots in
csrc/nks_internal.h) cover every (site block, job) pair exactly once and
never map a workgroup outside the rectangle, for every map, block count and
job count a call can have up to the sizes checked.  Host code only (the
header's functions are host/device), compiled with hipcc; no GPU needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0912_4457_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <vector>
#include "nks_internal.h"
int main() {
    long checked = 0;
    for (int xm = 1; xm <= 3; ++xm)
        for (int nb = 1; nb <= 300; nb += (nb < 40 ? 1 : 7))
            for (int nj = 1; nj <= 70; ++nj) {
                std::vector<int> hit((size_t)nb * nj, 0);
                const int grid = 8 * nks::xcd_slots(nb, nj, xm);
                for (int b = 0; b < grid; ++b) {
                    int sb = -1, job = -1;
                    if (!nks::map_block(b, nb, nj, xm, sb, job)) continue;
                    if (sb < 0 || sb >= nb || job < 0 || job >= nj) {
                        std::printf("OUT xm=%d nb=%d nj=%d b=%d sb=%d job=%d\n", xm, nb, nj, b, sb, job);
                        return 1;
                    }
                    hit[(size_t)sb * nj + job] += 1;
                }
                for (size_t q = 0; q < hit.size(); ++q)
                    if (hit[q] != 1) {
                        std::printf("COVER xm=%d nb=%d nj=%d pair=%zu hits=%d\n", xm, nb, nj, q, hit[q]);
                        return 1;
                    }
                ++checked;
            }
    std::printf("ok %ld\n", checked);
    return 0;
}
"""


def test_launch_maps_are_bijections(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "map.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "map"
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-I", CSRC, "-o", str(exe), str(src)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    assert out.stdout.startswith("ok ")
