"""Host side of the specialised tile-pass kernels: the generated source of a
pass compiles for gfx950 with the ROCm device compiler (no GPU needed),
without scratch spills and with at least two waves per SIMD; its structure
follows the pass record (one register-body call per fused gate)."""
import os
import re
import shutil
import subprocess

import pytest

import paper_2303_00123_amd as q
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = os.environ.get("QSV_JIT_CLANG", os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"),
                                                     "llvm", "bin", "clang++"))
HEADERS = [os.path.join(ROOT, "include", "qsv.h")] + [
    os.path.join(ROOT, "paper_2303_00123_amd", "csrc", f)
    for f in ("qsv_common.h", "qsv_internal.h", "qsv_tile_core.h")]


def test_generated_source_follows_the_plan():
    c = W.layered_cnot_brick(20, 4, seed=850)
    recs, pas = q.plan_fused(c.n, c.gates, c.params, q.QSV_C128)
    src = q.jit_source(c.n, c.gates, int(pas[0]))
    calls = re.findall(r"\brg_(1q|1d|1r|c1q|cx|cd|2q)<", src)
    # every fused gate of the pass that runs is one call; trailing
    # permutation gates are folded into the write offsets
    n_pass = int((pas == pas[0]).sum())
    assert 0 < len(calls) <= n_pass
    assert "switch" not in src


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no ROCm device compiler")
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_generated_source_compiles_without_spills(tmp_path, dtype):
    dt = q.QSV_C128 if dtype == "c128" else q.QSV_C64
    c = W.layered_cnot_brick(30, 20, seed=3002)
    for h in HEADERS:
        shutil.copy(h, tmp_path)
    src = tmp_path / "pass.hip"
    src.write_text(q.jit_source(c.n, c.gates, 2, dtype=dt))
    r = subprocess.run([CLANG, "-x", "hip", "--offload-arch=gfx950", "--cuda-device-only",
                        "--no-gpu-bundle-output", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops", "-Rpass-analysis=kernel-resource-usage",
                        "-I", str(tmp_path), str(src), "-o", str(tmp_path / "pass.co")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    scratch = int(re.search(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr).group(1))
    occ = int(re.search(r"Occupancy \[waves/SIMD\]: (\d+)", r.stderr).group(1))
    assert scratch <= 64 and occ >= 2


def test_stage_search_keeps_lds_exchanges_low():
    """Register stages take their bits by search (the addition after which
    the stage holds the most gates), not by an in-order fill, and the last
    two stages are re-split so that no empty store stage is needed: on the
    30-qubit brick the 20 passes need at most 364 LDS barriers (4 per split
    stage change, 3 for the first); an in-order fill needed 464."""
    c = W.layered_cnot_brick(30, 20, seed=3002)
    recs, pas = q.plan_fused(c.n, c.gates, c.params, q.QSV_C128)
    npass = int(pas.max()) + 1
    assert npass == 20
    barriers = sum(q.jit_source(c.n, c.gates, p, params=c.params).count("lds_barrier")
                   for p in range(npass))
    assert barriers <= 364
