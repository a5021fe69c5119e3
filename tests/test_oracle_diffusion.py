"""Pins of the oracle's mixture-averaged diffusion coefficients (CPU only).

Section 2 names mixture-averaged diffusion with Takahashi's high-pressure correction; the
chart behind that correction is not available here, so the oracle (and the library) give
the low-pressure Chapman-Enskog result, pinned below against the textbook collision
integral table, the textbook Chapman-Enskog constant, measured binary coefficients and the
trace limit of the mixture rule.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ATM = 101325.0


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def sp8():
    return synth.load_species(synth.FLAME_SPECIES)


def test_neufeld_diffusion_collision_integral_against_lj_table(orc):
    tab = gold("textbook_values.json")["lj_omega11"]
    for k, v in tab.items():
        if not k.startswith("_"):
            assert orc.omega_d(float(k)) == pytest.approx(v, rel=2e-3), k


def test_chapman_enskog_prefactor_is_the_textbook_constant(orc):
    """D * p * sigma^2 * Omega_D / sqrt(T^3 (1/MA + 1/MB)) in cm^2/s, atm, Angstrom, g/mol.
    The textbook's 0.0018583 predates the exact 2019 values of k_B and N_A, with which the
    same expression is 0.0018588: 3e-4 apart."""
    c = gold("textbook_values.json")["chapman_enskog_constant"]["value"]
    T, MA, MB, sig, eps = 420.0, 0.044, 0.002, 3.2e-10, 150.0
    D = orc.binary_diffusion(T, ATM, MA, MB, sig, eps)           # m^2/s at 1 atm
    got = D * 1e4 * (sig * 1e10) ** 2 * orc.omega_d(T / eps) / math.sqrt(T ** 3 * (1 / (MA * 1e3) + 1 / (MB * 1e3)))
    assert got == pytest.approx(c, rel=4e-4)


def test_pressure_and_temperature_scaling(orc):
    """D is proportional to 1/P, and to T^1.5 / Omega_D(T*)."""
    a = orc.binary_diffusion(500.0, 1e5, 0.028, 0.032, 3.5e-10, 110.0)
    b = orc.binary_diffusion(500.0, 1e7, 0.028, 0.032, 3.5e-10, 110.0)
    assert a / b == pytest.approx(100.0, rel=1e-14)
    c = orc.binary_diffusion(1000.0, 1e5, 0.028, 0.032, 3.5e-10, 110.0)
    ratio = (1000.0 / 500.0) ** 1.5 * orc.omega_d(500.0 / 110.0) / orc.omega_d(1000.0 / 110.0)
    assert c / a == pytest.approx(ratio, rel=1e-14)


def test_measured_binary_coefficients(orc, sp8):
    """Chung's corresponding-states Lennard-Jones parameters against measured values at
    1 atm (loose: the relations are not fitted to diffusion data)."""
    names = [s["name"] for s in sp8]
    for key, ref in gold("textbook_values.json")["measured_binary_diffusion_1atm"].items():
        if key.startswith("_"):
            continue
        a, b, T = key.split("|")
        T = float(T)
        i, j = names.index(a), names.index(b)
        Y = np.zeros((8, 1))
        Wi, Wj = sp8[i]["W"], sp8[j]["W"]
        Y[i] = 1e-12 * Wi
        Y[j] = 1.0 - Y[i]
        D = orc.Mech(sp8).mixdiff([ATM], [T], Y)[i, 0] * 1e4         # trace i in j
        assert D == pytest.approx(ref, rel=0.2), (key, D)


def test_trace_species_limit_is_the_binary_coefficient(orc, sp8):
    """A trace species in a pure bath diffuses with the binary coefficient of the pair,
    whatever the bath: D_i -> D_ij as Y_i -> 0 and X_j -> 1."""
    m = orc.Mech(sp8)
    for i, j in ((0, 1), (5, 3), (2, 7)):
        Y = np.zeros((8, 2))
        Y[i], Y[j] = 1e-14, 1.0 - 1e-14
        Y[:, 1] = 0.0
        Y[j, 1] = 0.5
        Y[i, 1] = 0.5
        D = m.mixdiff([2e6, 2e6], [900.0, 900.0], Y)
        # the binary coefficient from the 50/50 mixture: D_i = (1 - Y_i) D_ij / X_j
        W = np.array([s["W"] for s in sp8])
        X = (Y[:, 1] / W) / (Y[:, 1] / W).sum()
        Dij = D[i, 1] * X[j] / (1 - Y[i, 1])
        assert D[i, 0] == pytest.approx(Dij, rel=1e-12)
        # and it is symmetric
        Dji = D[j, 1] * X[i] / (1 - Y[j, 1])
        assert Dij == pytest.approx(Dji, rel=1e-13)


def test_single_species_has_zero_mixture_coefficient(orc, sp8):
    Y = np.zeros((8, 1))
    Y[1] = 1.0
    D = orc.Mech(sp8).mixdiff([1e7], [300.0], Y)
    assert D[1, 0] == 0.0 and np.all(np.isfinite(D))
