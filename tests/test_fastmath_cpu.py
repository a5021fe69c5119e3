"""Host build of the kernels' double-precision log, exp and table exp (fastmath.hpp): error in units of the
last place against long-double libm over seeded arguments (CPU only; the device build runs
the same arithmetic, and the GPU parity tests cover it end to end)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("fm") / "fmcheck")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "native", "fastmath_check.cpp")])
    out = subprocess.check_output([exe], text=True)
    kv = {}
    for line in out.splitlines():
        parts = line.split()
        for k, v in zip(parts[::2], parts[1::2]):
            kv[k] = float(v)
    return kv


def test_log_within_two_ulp(report):
    assert report["log_max_ulp"] <= 2.0


def test_log_of_non_positive_is_nan(report):
    assert report["log_neg_nan"] == 1 and report["log_zero_nan"] == 1


def test_exp_within_two_ulp(report):
    assert report["exp_max_ulp"] <= 2.0
    assert report["exp_sub_max_denorm_ulp"] <= 1.0


def test_exp_limits(report):
    assert report["exp_under_zero"] == 1 and report["exp_over_inf"] == 1
    assert report["exp_nan"] == 1 and report["exp_zero_one"] == 1


def test_table_exp_within_two_ulp(report):
    """exp_tab with its table of 2^(j/64): the transport and diffusion exponentials."""
    assert report["exptab_max_ulp"] <= 2.0
    assert report["exptab_sub_max_denorm_ulp"] <= 1.0
    assert report["exptab_limits"] == 1
