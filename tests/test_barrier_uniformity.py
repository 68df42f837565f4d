"""The team barriers of the ant kernel sit in uniform control flow.

CPU only: compiles one ant kernel with 8 waves per ant to LLVM IR for gfx950,
runs LLVM's uniformity analysis and checks that no workgroup barrier lies in
the region of a divergent branch (where it could execute with an empty exec
mask and pair the team's commands wrongly).  The checker itself is pinned on a
small kernel with a barrier under a lane-dependent branch, which it must
flag, and the same barrier under a uniform branch, which it must not."""
import os
import subprocess

import pytest

from tests.barrier_uniformity import check

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
OPT = "/opt/rocm/llvm/bin/opt"
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "--cuda-device-only", "-S", "-emit-llvm"]

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(OPT)),
                                reason="ROCm compiler not found")


def _uniformity(src, tmp_path):
    hip = tmp_path / "k.hip"
    hip.write_text(src)
    ll = tmp_path / "k.ll"
    subprocess.run([HIPCC, *FLAGS, str(hip), "-o", str(ll)], check=True,
                   capture_output=True)
    r = subprocess.run([OPT, "-mtriple=amdgcn-amd-amdhsa", "-mcpu=gfx950",
                        "-passes=print<uniformity>", "-disable-output", str(ll)],
                       capture_output=True, text=True, check=True)
    return check(r.stderr)


TOY = """
#include <hip/hip_runtime.h>
__global__ void toy(int *p, int n) {
  p[threadIdx.x] = 1;
  if (%s) __syncthreads();
  p[threadIdx.x + 64] = 2;
}
"""


def test_checker_flags_lane_dependent_barrier(tmp_path):
    st, bad = _uniformity(TOY % "threadIdx.x < (unsigned)n", tmp_path)
    assert st["barriers"] == 1 and len(bad) == 1


def test_checker_accepts_uniform_barrier(tmp_path):
    st, bad = _uniformity(TOY % "n > 3", tmp_path)
    assert st["barriers"] == 1 and bad == []


@pytest.mark.parametrize("inst", [
    "template __global__ void faco::ant_kernel<16, 8>(faco::Inst, int);",
    # the same kernel on segment-list tours (team moves and materialisations)
    "template __global__ void faco::ant_kernel<16, 8, true>(faco::Inst, int);",
    # the persistent batched kernel: dispatch loop, ant, update, all on barriers
    "template __global__ void faco::ant_persist_kernel<16, 8>(const faco::Inst *, "
    "faco::BatchCtl *, faco::BatchRun *, int);",
])
def test_team_barriers_in_uniform_control_flow(tmp_path, inst):
    kern = os.path.join(ROOT, "paper_2203_02228_amd", "csrc", "faco_kernels.hpp")
    st, bad = _uniformity(f'#include "{kern}"\n{inst}\n', tmp_path)
    assert st["barriers"] >= 20, st
    assert bad == [], f"barriers under divergent branches: {bad[:4]}"
