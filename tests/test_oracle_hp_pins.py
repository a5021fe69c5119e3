"""Pins of the oracle's (h, P, Y) state and of the extra solver outputs (CPU only).

The pressure-based solver refreshes its properties from enthalpy and pressure in every
pressure-correction loop (Section 3) and its surrogate outputs include psi = d rho/d p at
constant enthalpy, the thermal diffusivity and the species' nondimensional standard-state
enthalpies (Section 4.1).  Each is checked here against something other than its own
formula: round trips through the (P, T, Y) state, finite differences along an isenthalp,
ideal-gas closed forms, the formation enthalpies the NASA fits were built on, and the
Eucken/Chapman-Enskog Prandtl number of a monatomic gas.
"""
import numpy as np
import pytest

import synth

R = 8.31446261815324


@pytest.fixture(scope="module")
def sp8():
    return synth.load_species(synth.FLAME_SPECIES)


@pytest.fixture(scope="module")
def mech8(orc, sp8):
    return orc.Mech(sp8, synth.synthetic_kij(8))


def _h_tol(a):
    """Relative T resolution of a converged (h, P) bisection: |dh| ~ ulp(h_scale)."""
    return 4e-12 * np.maximum(1.0, a["h_scale"] / (a["T"] * np.abs(a["cp"])))


# ---------------------------------------------------------------------------------------
# (h, P, Y) -> T
# ---------------------------------------------------------------------------------------

def test_hp_round_trip_flame_field(orc, mech8):
    P, T, Y = synth.flame_field(16, seed=4)
    a = mech8.state_PT(P, T, Y, transport=False)
    b = mech8.state_hP(a["h"], P, Y, transport=False)
    assert np.all(b["status"] & (orc.NONPHYS | orc.BRACKET) == 0)
    assert np.all(np.abs(b["T"] / T - 1) <= _h_tol(a))
    assert np.all(b["P"] == P)
    assert np.max(np.abs(b["rho"] / a["rho"] - 1)) < 1e-9
    assert np.max(np.abs(b["h"] - a["h"]) / a["h_scale"]) < 1e-14


def test_hp_round_trip_two_species_cells(orc):
    P, T, Y = synth.cells_uniform(256, seed=31)
    m = orc.Mech(synth.load_species(["CH4", "O2"]), [[0, 0.03], [0.03, 0]])
    a = m.state_PT(P, T, Y, transport=False)
    b = m.state_hP(a["h"], P, Y, transport=False)
    ok = a["status"] & orc.NONPHYS == 0
    assert ok.sum() > 200
    assert np.all(np.abs(b["T"] / T - 1)[ok] <= _h_tol(a)[ok])


def test_hp_bracket_and_nonphysical_flags(orc, mech8):
    Y = np.zeros((8, 6))
    Y[1] = 1.0
    P = np.array([10e6, 10e6, -1.0, 10e6, 10e6, 10e6])
    h = np.array([5e7, -5e7, 0.0, 0.0, np.nan, 0.0])
    Y[:, 5] = 0.0
    Y[1, 5] = 0.9
    r = mech8.state_hP(h, P, Y, transport=False)
    assert r["status"][0] & orc.BRACKET and r["status"][1] & orc.BRACKET
    assert r["status"][2] & orc.NONPHYS and r["status"][4] & orc.NONPHYS
    assert r["status"][5] & orc.NONPHYS
    assert r["status"][3] == 0 and np.isfinite(r["T"][3])
    assert np.all(np.isnan(r["T"][[0, 1, 2, 4, 5]]))


def test_hp_in_the_enthalpy_gap_ends_at_the_root_switch(orc):
    """Pure O2 below its critical pressure: h(T; P) jumps where the Gibbs-selected root
    switches from liquid- to vapour-like.  An h* inside the jump has no solution; the
    bisection ends at the switch temperature, with a liquid-like root just below it and a
    vapour-like root just above it."""
    m = orc.Mech(synth.load_species(["O2"]))
    P = 3.0e6
    T = np.linspace(100.0, 150.0, 501)
    s = m.state_PT(np.full(T.size, P), T, np.ones((1, T.size)), transport=False)
    k = int(np.argmax(np.diff(s["Z"])))          # the jump of Z
    hl, hv = s["h"][k], s["h"][k + 1]
    assert hv - hl > 5e4                         # a latent heat, J/kg
    r = m.state_hP([0.5 * (hl + hv)], [P], [[1.0]], transport=False)
    Ts = r["T"][0]
    assert T[k] <= Ts <= T[k + 1]
    lo = m.state_PT([P], [Ts * (1 - 1e-9)], [[1.0]], transport=False)
    hi = m.state_PT([P], [Ts * (1 + 1e-9)], [[1.0]], transport=False)
    assert lo["Z"][0] < 0.3 < hi["Z"][0]


# ---------------------------------------------------------------------------------------
# psi = (d rho / d P) at constant h
# ---------------------------------------------------------------------------------------

def test_psi_by_finite_differences_along_the_isenthalp(orc, mech8):
    """Central difference of rho(h*, P) from the (h, P, Y) inversion itself."""
    P, T, Y = synth.flame_field(8, seed=12)
    a = mech8.state_PT(P, T, Y, transport=False)
    d = 1e-4 * P
    rp = mech8.state_hP(a["h"], P + d, Y, transport=False)
    rm = mech8.state_hP(a["h"], P - d, Y, transport=False)
    fd = (rp["rho"] - rm["rho"]) / (2 * d)
    assert np.max(np.abs(fd / a["psi"] - 1)) < 1e-6


def test_psi_by_finite_differences_two_species(orc):
    P, T, Y = synth.cells_uniform(64, seed=33)
    m = orc.Mech(synth.load_species(["CH4", "O2"]), [[0, 0.03], [0.03, 0]])
    a = m.state_PT(P, T, Y, transport=False)
    d = 1e-5 * P
    rp = m.state_hP(a["h"], P + d, Y, transport=False)
    rm = m.state_hP(a["h"], P - d, Y, transport=False)
    smooth = (rp["nphys"] == a["nphys"]) & (rm["nphys"] == a["nphys"]) & (a["nphys"] == 1)
    fd = (rp["rho"] - rm["rho"]) / (2 * d)
    assert smooth.sum() > 30
    assert np.max(np.abs(fd / a["psi"] - 1)[smooth]) < 1e-5


@pytest.mark.parametrize("T", [150.0, 800.0, 2800.0])
def test_psi_ideal_gas_limit(mech8, sp8, T):
    """Ideal gas: h = h(T), so (d rho/d P)_h = (d rho/d P)_T = W/(R T) = rho/P; and
    c^2 = gamma P/rho, so psi = gamma / c^2."""
    rng = np.random.default_rng(int(T))
    Y = rng.dirichlet(np.ones(8), 5).T
    r = mech8.state_PT(np.full(5, 1.0), np.full(5, T), Y, transport=False)
    W = 1.0 / np.sum(Y / np.array([s["W"] for s in sp8])[:, None], axis=0)
    assert np.allclose(r["psi"], W / (R * T), rtol=1e-6)
    gamma = r["cp"] / r["cv"]
    assert np.allclose(r["psi"], gamma / r["c"] ** 2, rtol=1e-6)


# ---------------------------------------------------------------------------------------
# h_i/(R T) and the thermal diffusivity
# ---------------------------------------------------------------------------------------

def test_species_hRT_at_298_is_the_formation_enthalpy(mech8, sp8):
    r = mech8.state_PT([1.0], [298.15], np.full((8, 1), 1 / 8), transport=False)
    for i, s in enumerate(sp8):
        assert r["hRT"][0, i] * R * 298.15 == pytest.approx(s["dhf298"], abs=1e-6 * 1e5)
    assert np.all(r["hRT"][0, 8:] == 0.0)


@pytest.mark.parametrize("T", [200.0, 700.0, 1500.0, 3000.0])
def test_species_hRT_derivative_is_the_species_cp(orc, sp8, T):
    """d(R T h_i/RT)/dT = c_p,i, with c_p,i from a one-species mechanism's ideal part."""
    m8 = orc.Mech(sp8)
    d = 1e-4 * T
    Y = np.full((8, 1), 1 / 8)
    hp = m8.state_PT([1.0], [T + d], Y, transport=False)["hRT"][0, :8] * (T + d)
    hm = m8.state_PT([1.0], [T - d], Y, transport=False)["hRT"][0, :8] * (T - d)
    fd = (hp - hm) / (2 * d)
    for i, s in enumerate(sp8):
        cp_i = orc.Mech([s]).state_PT([1.0], [T], [[1.0]], transport=False)["cp_ig"][0] * s["W"] / R
        assert fd[i] == pytest.approx(cp_i, rel=1e-7)


def test_mixture_ideal_enthalpy_is_the_mass_weighted_species_sum(mech8, sp8):
    P, T, Y = synth.flame_field(6, seed=2)
    r = mech8.state_PT(P, T, Y, transport=False)
    W = np.array([s["W"] for s in sp8])
    h = np.sum(Y * (R * T / W[:, None]) * r["hRT"][:, :8].T, axis=0)
    assert np.max(np.abs(h - r["h_ig"]) / r["h_scale"]) < 1e-13


def test_alpha_gives_the_monatomic_prandtl_number(orc):
    """A monatomic dilute gas (c_p = 5/2 R, no internal modes) has the Chapman-Enskog
    Prandtl number nu/alpha = 2/3; Chung's 31.2 vs 15/4 R = 31.18 allows 1e-3."""
    ar = {"name": "Ar", "W": 0.039948, "Tc": 150.86, "Pc": 4.898e6, "Vc": 74.57e-6,
          "omega": -0.002, "dipole": 0.0, "kappa": 0.0, "Tmid": 1000.0,
          "nasa_lo": [2.5, 0, 0, 0, 0, -745.375, 4.37967], "nasa_hi": [2.5, 0, 0, 0, 0, -745.375, 4.37967]}
    m = orc.Mech([ar])
    T = np.array([300.0, 1000.0, 2500.0])
    r = m.state_PT(np.full(3, 100.0), T, np.ones((1, 3)))
    Pr = (r["mu"] / r["rho"]) / r["alpha"]
    assert np.allclose(Pr, 2.0 / 3.0, rtol=1.5e-3)


def test_alpha_is_nan_without_transport(mech8):
    r = mech8.state_PT([10e6], [300.0], np.full((8, 1), 1 / 8), transport=False)
    assert np.isnan(r["alpha"][0]) and np.isfinite(r["psi"][0])
