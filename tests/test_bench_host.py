"""Host-side checks of bench.py: the per-particle byte counts behind its
roofline figures, and the one-GPU contract.  No GPU is used."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("dim,q,calls", [(2, False, 152), (2, True, 176), (3, False, 224)])
def test_three_call_bytes_fp64(dim, q, calls):
    """Three calls: gather_push reads and writes x, v and writes a 4-byte bin;
    the rebin reads the bins and reads and writes every record; the deposit
    reads the positions (and charges)."""
    assert bench.algorithmic_bytes(dim, q)["calls"] == calls


@pytest.mark.parametrize("dim,calls", [(2, 80), (3, 116)])
def test_three_call_bytes_fp32(dim, calls):
    assert bench.algorithmic_bytes_f32(dim, False)["calls"] == calls


def test_fused_bytes_per_pass_form():
    """2D FP64: key pass 36, group pass 8, writing pass 68, deposit 16."""
    ab = bench.algorithmic_bytes(2, False)
    assert (ab["step_key"], ab["step_group"], ab["step_emit"], ab["deposit_bins"]) == (36, 8, 68, 16)
    assert ab["fused"] == 128
    # the fused step moves fewer bytes than the three calls
    for dim in (2, 3):
        for q in (False, True):
            ab = bench.algorithmic_bytes(dim, q)
            assert ab["fused"] < ab["calls"]


def test_fused_bytes_with_the_writing_pass_deposit():
    """When the writing pass deposits, the deposit reads no positions: the 2D
    step moves 112 B (key 36, group 8, writing 68)."""
    ab = bench.algorithmic_bytes(2, False, emit_deposit=True)
    assert ab["fused"] == 112
    assert ab["step_emit"] == bench.algorithmic_bytes(2, False)["step_emit"]
    # with the key pass and the ranking in one kernel no keys are written or read
    assert bench.algorithmic_bytes(2, False, emit_deposit=True, fused_rank=True)["fused"] == 104


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


@pytest.mark.parametrize("dim,level", [(2, 2), (2, 3), (3, 2)])
def test_bench_poisson_solve_equals_the_oracle_support(dim, level):
    """The benchmark's field solve (Langmuir support, outside the hot path)
    equals the oracle's periodic Poisson solve and central-difference field,
    which the oracle's cold-plasma and Bohm-Gross pins fix."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(dim * 10 + level)
    n = 3 ** (dim * level)
    rho = -(1.0 + 0.05 * rng.standard_normal(n)) / n
    E_b = bench.poisson_field(rho, dim, level)
    E_o = oracle.field_from_potential(oracle.poisson_periodic(rho, dim, level), dim, level)
    assert np.abs(E_b - E_o).max() <= 1e-12 * np.abs(E_o).max()
