"""CPU check of the matrix-core operand tables (no GPU).

tests/mfma_emul.cpp builds the FP16 high/low tables with the library's host
code and runs the kernel's dataflow through a software model of
v_mfma_f32_16x16x16_f16 (lane layout as documented in plan_internal.h); the
trajectory evaluation, the sums N^T g and the xi-update must match FP64 to
about 22 significant bits. tests/mfma32_emul.cpp does the same for the FP32
form (v_mfma_f32_16x16x4f32, the lane-group transpose by permlane swaps,
FP32 tables): FP32 accuracy."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_02224_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _build(tmp_path_factory, name):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("mfma") / name)
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(ROOT, "tests", name + ".cpp"), os.path.join(CSRC, "precompute.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


@pytest.fixture(scope="module")
def emul(tmp_path_factory):
    return _build(tmp_path_factory, "mfma_emul")


@pytest.fixture(scope="module")
def emul32(tmp_path_factory):
    return _build(tmp_path_factory, "mfma32_emul")


@pytest.mark.parametrize("T,M", [(100, 10), (50, 4), (128, 20), (16, 0), (37, 3)])
def test_operand_tables_reproduce_fp64_products(emul, T, M):
    r = subprocess.run([emul, str(T), str(M)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("T,M", [(100, 20), (50, 4), (128, 10), (16, 0), (37, 3)])
def test_fp32_operand_tables_reproduce_fp64_products(emul32, T, M):
    r = subprocess.run([emul32, str(T), str(M)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
