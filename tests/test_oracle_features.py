"""Pins of the surrogate-feature oracle (CPU only): Bilger's mixture fraction and the
Box-Cox transform of the paper's (h, p, Z) inputs (Sections 4.1-4.2)."""
import numpy as np
import pytest

import synth
from oracle import features as of


@pytest.fixture(scope="module")
def sp8():
    return synth.load_species(synth.FLAME_SPECIES)


def test_pure_streams(sp8):
    Y = np.eye(8)
    Z = of.bilger_Z(sp8, Y, fuel=0, oxidizer=1)
    assert Z[0] == pytest.approx(1.0, abs=1e-15) and Z[1] == pytest.approx(0.0, abs=1e-15)


def test_unburnt_mixing_line_is_exact(sp8):
    """beta is linear in Y, so a mix of the two streams has Z equal to its fuel fraction."""
    xi = np.linspace(0.0, 1.0, 101)
    Y = np.zeros((8, xi.size))
    Y[0], Y[1] = xi, 1.0 - xi
    assert np.max(np.abs(of.bilger_Z(sp8, Y, 0, 1) - xi)) < 1e-14


def test_burke_schumann_products_conserve_the_mixture_fraction(sp8):
    """Complete combustion CH4 + 2 O2 -> CO2 + 2 H2O conserves elements, so the burnt
    Burke-Schumann state of mixture fraction xi has Bilger Z = xi (to the consistency of
    the tabulated molar masses with the atomic masses, ~1e-4)."""
    W = {s["name"]: s["W"] for s in sp8}
    xst = W["CH4"] / (W["CH4"] + 2 * W["O2"])
    yco2 = W["CO2"] / (W["CO2"] + 2 * W["H2O"])
    xi = np.linspace(0.0, 1.0, 201)
    lean = xi <= xst
    prod = np.where(lean, xi / xst, (1 - xi) / (1 - xst))
    Y = np.zeros((8, xi.size))
    Y[0] = np.where(lean, 0.0, (xi - xst) / (1 - xst))
    Y[1] = np.where(lean, 1 - xi / xst, 0.0)
    Y[2] = yco2 * prod
    Y[3] = (1 - yco2) * prod
    Z = of.bilger_Z(sp8, Y, 0, 1)
    assert np.max(np.abs(Z - xi)) < 2e-4
    assert of.bilger_Z(sp8, Y[:, [np.argmin(np.abs(xi - xst))]], 0, 1)[0] == pytest.approx(xst, abs=3e-3)


def test_hydrogen_and_water_have_consistent_weights(sp8):
    """OH and H2O differ by one H: their coupling functions per mole differ by 1/2."""
    mol = {s["name"]: s for s in sp8}
    b = lambda name: of.coupling_beta(sp8, np.eye(8)[:, [list(mol).index(name)]])[0] * mol[name]["W"]  # noqa: E731
    assert b("H2O") - b("OH") == pytest.approx(0.5, abs=2e-3)
    assert b("CH4") == pytest.approx(2 + 2, abs=5e-3) and b("O2") == pytest.approx(-2, abs=5e-3)


@pytest.mark.parametrize("lam", [0.1, 0.25, 0.5, 1.0])
def test_box_cox_closed_forms(lam):
    Z = np.array([0.0, 1.0, 0.25, -1e-9])
    bc = of.box_cox(Z, lam)
    assert bc[0] == pytest.approx(-1 / lam) and bc[1] == pytest.approx(0.0, abs=1e-15)
    assert bc[2] == pytest.approx((0.25 ** lam - 1) / lam, rel=1e-15)
    assert bc[3] == bc[0]                                  # clamped at 0
    # lambda -> 0 tends to the logarithm
    assert of.box_cox(np.array([0.3]), 1e-7)[0] == pytest.approx(np.log(0.3), rel=1e-5)


def test_box_cox_rejects_lambda_zero():
    with pytest.raises(ValueError):
        of.box_cox(np.array([0.5]), 0.0)
