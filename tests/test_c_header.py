"""The boundary from C: a C99 program that includes include/gmc.h, links libgmc.so and uses
its host-only calls (plan, workspace size, launch configuration, argument errors). No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_2401_09283_amd")

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "gmc.h"

int main(void) {
    gmc_geometry g;
    memset(&g, 0, sizeof g);
    g.n_views = 10; g.det_w = 64; g.det_h = 48;
    g.nx = 20; g.ny = 18; g.nz = 17;
    g.voxel_mm[0] = g.voxel_mm[1] = g.voxel_mm[2] = 1.0;
    g.origin_mm[0] = -9.5; g.origin_mm[1] = -8.5; g.origin_mm[2] = -8.0;
    g.weighting = GMC_WEIGHT_FDK; g.grad_mode = GMC_GRAD_PAPER; g.flags = 0;
    gmc_plan* plan = NULL;
    if (gmc_plan_create(&g, NULL, &plan) != GMC_OK || !plan) { printf("create failed: %s\n", gmc_last_error()); return 1; }
    int64_t info[8];
    if (gmc_plan_info(plan, info) != GMC_OK) return 2;
    size_t ws = gmc_workspace_bytes(plan);
    printf("brick %lld %lld %lld bricks %lld ws %zu\n", (long long)info[0], (long long)info[1], (long long)info[2],
           (long long)info[5], ws);
    /* argument errors come back as status codes with a message, before any launch */
    gmc_status st = gmc_bp_forward(plan, NULL, NULL, NULL, NULL);
    printf("null args -> %d (%s)\n", (int)st, gmc_last_error());
    g.n_views = 0;
    gmc_plan* bad = NULL;
    st = gmc_plan_create(&g, NULL, &bad);
    printf("empty geometry -> %d (%s)\n", (int)st, gmc_status_string(st));
    gmc_plan_destroy(plan);
    return (st == GMC_E_INVALID && bad == NULL) ? 0 : 3;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a C compiler")
def test_c_program_uses_the_abi(tmp_path):
    lib = os.path.join(LIB_DIR, "libgmc.so")
    if not os.path.exists(lib):
        pytest.skip("libgmc.so is not built")
    src = tmp_path / "use_gmc.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "use_gmc"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-L", LIB_DIR, "-lgmc", "-Wl,-rpath," + LIB_DIR, "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.splitlines()
    assert lines[0].startswith("brick 16 16 16 bricks 8 ws ")
    assert lines[1].startswith("null args -> %d (workspace is NULL" % -2)   # the workspace is checked first
    assert lines[2].startswith("empty geometry -> %d" % -1)
