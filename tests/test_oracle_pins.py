"""Pins of the CPU oracle against what the paper and mathematics fix (CPU only).

Every test here checks the oracle against something other than itself: values the paper
prints (tests/golden/paper_values.json), textbook tables, closed forms, exact identities,
brute force, finite differences, and reductions to simpler cases.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
R = 8.31446261815324


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def sp8():
    return synth.load_species(synth.FLAME_SPECIES)


@pytest.fixture(scope="module")
def mech8(orc, sp8):
    return orc.Mech(sp8, synth.synthetic_kij(8))


@pytest.fixture(scope="module")
def mech8_k0(orc, sp8):
    return orc.Mech(sp8)


# ---------------------------------------------------------------------------------------
# Peng-Robinson constants and the critical point (Section 2, Eq. 1)
# ---------------------------------------------------------------------------------------

def test_exact_pr_constants_round_to_printed_values():
    """Derive Omega_a, Omega_b, Z_c from the critical conditions of Eq. (1) with mpmath;
    they must round to the paper's printed 0.45724 / 0.07780."""
    from mpmath import mp, mpf, findroot, diff
    mp.dps = 30

    def eqs(vc, b, a):
        P = lambda v: 1 / (v - b) - a / (v * v + 2 * b * v - b * b)  # noqa: E731 (R T_c = 1)
        return [diff(P, vc), diff(P, vc, 2), P(vc) - 1]

    vc, b, a = findroot(eqs, (mpf("0.31"), mpf("0.078"), mpf("0.457")))
    g = gold("paper_values.json")
    assert round(float(a), 5) == g["pr_omega_a_printed"]["value"]
    assert round(float(b), 5) == g["pr_omega_b_printed"]["value"]
    zc_closed = (11 - 2 * math.sqrt(7) * math.sinh(math.asinh(13 / (7 * math.sqrt(7))) / 3)) / 32
    assert abs(float(vc) - zc_closed) < 1e-14


@pytest.mark.parametrize("name", synth.FLAME_SPECIES[:6] + ("N2",))
def test_triple_root_at_critical_point(orc, name):
    """Pure fluid at (Tc, Pc): the cubic has a triple root at Z_c (closed form). A triple
    root is only accurate to ~eps^(1/3) in double precision, hence 1e-4."""
    s = synth.load_species([name])
    m = orc.Mech(s)
    r = m.state_PT([s[0]["Pc"]], [s[0]["Tc"]], [[1.0]], transport=False)
    zc = (11 - 2 * math.sqrt(7) * math.sinh(math.asinh(13 / (7 * math.sqrt(7))) / 3)) / 32
    assert abs(r["Z"][0] - zc) < 1e-4
    # the critical density follows from Z_c
    rho_c = s[0]["Pc"] * s[0]["W"] / (zc * R * s[0]["Tc"])
    assert abs(r["rho"][0] / rho_c - 1) < 1e-3


def test_rounded_constants_would_fail_the_critical_test():
    """Sanity of the pin itself: with the printed (rounded) constants, the cubic at
    (Tc, Pc) has a single real root near 0.3214, far from Z_c (the pin can fail)."""
    A, B = 0.45724, 0.07780
    roots = np.roots([1, -(1 - B), A - 3 * B * B - 2 * B, -(A * B - B * B - B ** 3)])
    real = roots[np.abs(roots.imag) < 1e-9].real
    assert len(real) == 1 and abs(real[0] - 0.32138) < 1e-4


def test_paper_critical_temperatures(sp8):
    g = gold("paper_values.json")
    tc = {s["name"]: s["Tc"] for s in sp8}
    assert round(tc["O2"]) in (g["Tc_O2_approx_K"]["value"], g["Tc_O2_approx_K"]["value"] + 1)
    assert round(tc["CH4"]) in (g["Tc_CH4_approx_K"]["value"], g["Tc_CH4_approx_K"]["value"] + 1)


# ---------------------------------------------------------------------------------------
# The cubic, its roots and Gibbs selection
# ---------------------------------------------------------------------------------------

def _eq1_pressure(Z, A, B):
    """Eq. (1) divided by P, with v = Z RT/P, a = A (RT)^2/P, b = B RT/P:
    1/(Z - B) - A/(Z^2 + 2BZ - B^2) - 1, which must vanish at every physical root."""
    return 1.0 / (Z - B) - A / (Z * Z + 2 * B * Z - B * B) - 1.0


@pytest.mark.parametrize("seed", range(5))
def test_cubic_roots_against_numpy_and_eq1(orc, seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(200):
        B = rng.uniform(0.001, 0.3)
        A = rng.uniform(0.0, 2.5)
        roots = orc.cubic_roots(A, B)
        ref = np.roots([1, -(1 - B), A - 3 * B * B - 2 * B, -(A * B - B * B - B ** 3)])
        # roots of a cubic with a near-double root are only known to ~sqrt(eps)
        real = np.sort(ref[np.abs(ref.imag) < 1e-6].real)
        if len(real) != len(roots):
            gaps = np.diff(np.sort(ref.real))
            assert np.min(np.abs(gaps)) < 1e-5 or np.min(np.abs(ref.imag)) < 1e-5
            continue
        np.testing.assert_allclose(roots, real, rtol=0, atol=1e-7)
        for z in roots:
            if z > B:  # physical roots satisfy Eq. (1) itself
                assert abs(_eq1_pressure(z, A, B)) < 1e-9 * (1 / (z - B) + 1 + A / abs(z * z + 2 * B * z - B * B))


def test_cubic_brute_force_root_count(orc):
    """Tiny inputs: count sign changes of Eq. (1) on a dense Z grid above B."""
    rng = np.random.default_rng(7)
    for _ in range(60):
        B = rng.uniform(0.01, 0.15)
        A = rng.uniform(0.05, 1.2)
        z = np.linspace(B * (1 + 1e-9), 1 + B, 200001)
        f = z * z * z - (1 - B) * z * z + (A - 3 * B * B - 2 * B) * z - (A * B - B * B - B ** 3)
        n_sc = int(np.sum(np.sign(f[1:]) != np.sign(f[:-1])))
        roots = [r for r in orc.cubic_roots(A, B) if r > B]
        assert len(roots) == n_sc


def test_f_at_B_is_negative(orc):
    """f(B) = -2 B^2 < 0, so a physical root above B always exists."""
    rng = np.random.default_rng(3)
    for _ in range(500):
        B = rng.uniform(1e-6, 0.5)
        A = rng.uniform(0.0, 5.0)
        roots = orc.cubic_roots(A, B)
        assert max(roots) > B


def _maxwell_psat(a, b, T):
    """Saturation pressure of a pure PR fluid by Maxwell's equal-area rule, computed with
    scipy quadrature and Brent's method straight from Eq. (1)."""
    from scipy.integrate import quad
    from scipy.optimize import brentq
    Pv = lambda v: R * T / (v - b) - a / (v * v + 2 * b * v - b * b)  # noqa: E731
    dP = lambda v: -R * T / (v - b) ** 2 + 2 * a * (v + b) / (v * v + 2 * b * v - b * b) ** 2  # noqa: E731
    vs = np.geomspace(b * 1.0001, b * 1e4, 200000)
    d = dP(vs)
    idx = np.where(np.sign(d[1:]) != np.sign(d[:-1]))[0]
    v_min = brentq(dP, vs[idx[0]], vs[idx[0] + 1])
    v_max = brentq(dP, vs[idx[1]], vs[idx[1] + 1])
    p_lo, p_hi = max(Pv(v_min), 1e3), Pv(v_max)

    def area(P):
        vl = brentq(lambda v: Pv(v) - P, b * (1 + 1e-12), v_min)
        vv = brentq(lambda v: Pv(v) - P, v_max, R * T / P * 10)
        return quad(lambda v: Pv(v) - P, vl, vv, limit=400, epsabs=0, epsrel=1e-11)[0]

    return brentq(area, p_lo * (1 + 1e-9), p_hi * (1 - 1e-9), xtol=1e-12, rtol=1e-14)


@pytest.mark.parametrize("name,T", [("O2", 120.0), ("CH4", 150.0)])
def test_gibbs_selection_switches_at_maxwell_psat(orc, name, T):
    s = synth.load_species([name])
    m = orc.Mech(s)
    am, _, _, bm = m.mix(np.array([1.0]), T)
    psat = _maxwell_psat(am, bm, T)
    below = m.state_PT([0.999 * psat], [T], [[1.0]], transport=False)
    above = m.state_PT([1.001 * psat], [T], [[1.0]], transport=False)
    assert below["nphys"][0] == 3 and above["nphys"][0] == 3
    assert below["status"][0] & orc.THREE_ROOT
    assert below["Z"][0] == pytest.approx(below["roots"][0][2], rel=1e-12)   # vapour
    assert above["Z"][0] == pytest.approx(above["roots"][0][0], rel=1e-12)   # liquid
    assert below["Z"][0] > 0.5 and above["Z"][0] < 0.1


def test_gibbs_energy_equal_at_maxwell_psat(orc):
    """At P_sat the two outer roots have equal residual Gibbs energy (Maxwell <=> Gibbs)."""
    s = synth.load_species(["O2"])
    m = orc.Mech(s)
    T = 120.0
    am, _, _, bm = m.mix(np.array([1.0]), T)
    psat = _maxwell_psat(am, bm, T)
    A = am * psat / (R * T) ** 2
    B = bm * psat / (R * T)
    r = orc.cubic_roots(A, B)
    assert len(r) == 3
    gl, gv = orc.gdep_RT(r[0], A, B), orc.gdep_RT(r[2], A, B)
    assert abs(gl - gv) < 1e-8


def test_gibbs_tie_flag_at_the_switch_pressure(orc):
    """Bisecting P for the root switch of pure O2 at 120 K ends at two adjacent doubles; there
    the two residual Gibbs energies agree to rounding, so the tie flag is set and the
    vapour-like root taken; a part in 1e6 away there is no tie.  The switch pressure is the
    Maxwell one."""
    s = synth.load_species(["O2"])
    m = orc.Mech(s)
    T = 120.0
    lo, hi = 1.0e6, 2.0e6                            # vapour-like at lo, liquid-like at hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid in (lo, hi):
            break
        z = m.state_PT([mid], [T], [[1.0]], transport=False)
        if z["Z"][0] > 0.3:
            lo = mid
        else:
            hi = mid
    assert np.nextafter(lo, np.inf) == hi
    at = m.state_PT([lo, hi], [T, T], [[1.0, 1.0]], transport=False)
    # the switch is the upper edge of the tie band: a tie (vapour-like root) below it,
    # the liquid-like root without a tie above it
    assert at["status"][0] & orc.GIBBS_TIE and at["Z"][0] > 0.3
    assert at["status"][1] & orc.GIBBS_TIE == 0 and at["Z"][1] < 0.3
    off = m.state_PT([lo * (1 - 1e-6), hi * (1 + 1e-6)], [T, T], [[1.0, 1.0]], transport=False)
    assert np.all(off["status"] & orc.GIBBS_TIE == 0)
    assert off["Z"][0] > 0.3 and off["Z"][1] < 0.3
    am, _, _, bm = m.mix(np.array([1.0]), T)
    assert lo == pytest.approx(_maxwell_psat(am, bm, T), rel=1e-9)


# ---------------------------------------------------------------------------------------
# Ideal-gas parts (NASA-7)
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("name", synth.FLAME_SPECIES)
def test_nasa_cp298_against_janaf(orc, name):
    s = synth.load_species([name])
    m = orc.Mech(s)
    r = m.state_PT([1.0], [298.15], [[1.0]], transport=False)
    cp_molar = r["cp_ig"][0] * s[0]["W"]
    ref = gold("textbook_values.json")["janaf_cp298_J_per_molK"][name]
    assert abs(cp_molar / ref - 1) < 0.02


@pytest.mark.parametrize("name", synth.FLAME_SPECIES)
def test_nasa_h298_is_formation_enthalpy_and_continuous(orc, name):
    s = synth.load_species([name])
    m = orc.Mech(s)
    r = m.state_PT([1.0], [298.15], [[1.0]], transport=False)
    assert r["h_ig"][0] * s[0]["W"] == pytest.approx(s[0]["dhf298"], abs=1e-6 * 1e5)
    lo = m.state_PT([1.0], [1000.0 * (1 - 1e-12)], [[1.0]], transport=False)
    hi = m.state_PT([1.0], [1000.0], [[1.0]], transport=False)
    assert hi["cp_ig"][0] == pytest.approx(lo["cp_ig"][0], rel=1e-9)
    assert hi["h_ig"][0] == pytest.approx(lo["h_ig"][0], rel=1e-9, abs=1e-3)


@pytest.mark.parametrize("T", [150.0, 500.0, 999.0, 1500.0, 2900.0])
def test_ideal_cp_is_dh_dT(mech8, T):
    Y = np.full((8, 1), 1 / 8)
    d = 1e-3 * T
    rp = mech8.state_PT([1.0], [T + d], Y, transport=False)
    rm = mech8.state_PT([1.0], [T - d], Y, transport=False)
    r0 = mech8.state_PT([1.0], [T], Y, transport=False)
    fd = (rp["h_ig"][0] - rm["h_ig"][0]) / (2 * d)
    assert fd == pytest.approx(r0["cp_ig"][0], rel=1e-6)


# ---------------------------------------------------------------------------------------
# Departures: ideal-gas limit and thermodynamic consistency
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("T", [130.0, 300.0, 1000.0, 2800.0])
def test_ideal_gas_limit(mech8, sp8, T):
    rng = np.random.default_rng(int(T))
    Y = rng.dirichlet(np.ones(8), 4).T
    r = mech8.state_PT(np.full(4, 1.0), np.full(4, T), Y, transport=False)
    W = 1.0 / np.sum(Y / np.array([s["W"] for s in sp8])[:, None], axis=0)
    assert np.all(np.abs(r["Z"] - 1) < 1e-6)
    assert np.all(np.abs(r["h"] - r["h_ig"]) < 1e-6 * r["h_scale"])
    assert np.all(np.abs(r["cp"] / r["cp_ig"] - 1) < 1e-6)
    gamma = r["cp_ig"] / (r["cp_ig"] - R / W)
    assert np.allclose(r["c"], np.sqrt(gamma * R * T / W), rtol=1e-6)
    assert np.allclose(r["rho"], 1.0 * W / (R * T), rtol=1e-6)


def _fd_states():
    P, T, Y = synth.cells_uniform(64, seed=21)
    sp = synth.load_species(["CH4", "O2"])
    return sp, P, T, Y


def test_cp_is_dh_dT_at_constant_P(orc):
    sp, P, T, Y = _fd_states()
    m = orc.Mech(sp, [[0, 0.03], [0.03, 0]])
    d = 1e-4 * T
    r0 = m.state_PT(P, T, Y, transport=False)
    rp = m.state_PT(P, T + d, Y, transport=False)
    rm = m.state_PT(P, T - d, Y, transport=False)
    same = (rp["nphys"] == 1) & (rm["nphys"] == 1) & (r0["nphys"] == 1)
    fd = (rp["h"] - rm["h"]) / (2 * d)
    rel = np.abs(fd / r0["cp"] - 1)[same]
    assert same.sum() > 50 and np.max(rel) < 2e-5


def test_cv_is_de_dT_at_constant_v(orc):
    sp, P, T, Y = _fd_states()
    m = orc.Mech(sp, [[0, 0.03], [0.03, 0]])
    r0 = m.state_PT(P, T, Y, transport=False)
    v = r0["v"]
    d = 1e-4 * T
    rp = m.state_vT(v, T + d, Y, transport=False)
    rm = m.state_vT(v, T - d, Y, transport=False)
    fd = (rp["e"] - rm["e"]) / (2 * d)
    assert np.max(np.abs(fd / r0["cv"] - 1)) < 1e-6


def test_sound_speed_from_isothermal_compressibility(orc):
    """c^2 = (cp/cv) (dP/drho)_T, with (dP/drho)_T by finite differences of Eq. (1)."""
    sp, P, T, Y = _fd_states()
    m = orc.Mech(sp, [[0, 0.03], [0.03, 0]])
    r0 = m.state_PT(P, T, Y, transport=False)
    v = r0["v"]
    d = 1e-6 * v
    rp = m.state_vT(v + d, T, Y, transport=False)
    rm = m.state_vT(v - d, T, Y, transport=False)
    dPdv = (rp["P"] - rm["P"]) / (2 * d)
    c2 = -(v * v / r0["W"]) * dPdv * r0["cp"] / r0["cv"]
    assert np.max(np.abs(np.sqrt(c2) / r0["c"] - 1)) < 1e-6


def test_dh_dP_maxwell_relation(orc):
    """(dh/dP)_T = v - T (dv/dT)_P (mass-specific), both sides by finite differences."""
    sp, P, T, Y = _fd_states()
    m = orc.Mech(sp)
    r0 = m.state_PT(P, T, Y, transport=False)
    dP = 1e-5 * P
    dT = 1e-5 * T
    hp = m.state_PT(P + dP, T, Y, transport=False)["h"]
    hm = m.state_PT(P - dP, T, Y, transport=False)["h"]
    vp = 1 / m.state_PT(P, T + dT, Y, transport=False)["rho"]
    vm = 1 / m.state_PT(P, T - dT, Y, transport=False)["rho"]
    lhs = (hp - hm) / (2 * dP)
    rhs = 1 / r0["rho"] - T * (vp - vm) / (2 * dT)
    ok = r0["nphys"] == 1
    assert np.max(np.abs(lhs - rhs)[ok] / np.abs(1 / r0["rho"][ok])) < 1e-4


@pytest.mark.parametrize("T", [200.0, 1500.0, 2500.0])
def test_am_derivatives_by_finite_differences(mech8, T):
    """Includes temperatures beyond T_r* where 1 + kappa(1 - sqrt(T_r)) < 0 for most
    species, so the sign-aware derivative of sqrt(a_i a_j) is exercised."""
    X = np.random.default_rng(1).dirichlet(np.ones(8))
    d = 1e-4 * T
    a0, a1, a2, _ = mech8.mix(X, T)
    ap = mech8.mix(X, T + d)[0]
    am = mech8.mix(X, T - d)[0]
    assert (ap - am) / (2 * d) == pytest.approx(a1, rel=1e-7)
    assert (ap - 2 * a0 + am) / (d * d) == pytest.approx(a2, rel=1e-4)
    a1p = mech8.mix(X, T + d)[1]
    a1m = mech8.mix(X, T - d)[1]
    assert (a1p - a1m) / (2 * d) == pytest.approx(a2, rel=1e-7)


# ---------------------------------------------------------------------------------------
# Mixing rules
# ---------------------------------------------------------------------------------------

def test_unit_composition_reduces_to_pure_species(orc, sp8, mech8):
    P = np.array([10e6, 5e6, 12e6])
    T = np.array([150.0, 800.0, 2500.0])
    for k, s in enumerate(sp8):
        Y = np.zeros((8, 3))
        Y[k] = 1.0
        a = mech8.state_PT(P, T, Y)
        b = orc.Mech([s]).state_PT(P, T, np.ones((1, 3)))
        for f in ("Z", "rho", "h", "cp", "c", "mu", "lambda"):
            np.testing.assert_allclose(a[f], b[f], rtol=1e-13, err_msg=f)


def test_k0_mixing_is_rank_one(orc, sp8, mech8_k0):
    X = np.random.default_rng(2).dirichlet(np.ones(8))
    for T in (150.0, 2000.0):
        sq = np.array([math.sqrt(orc.Mech([s]).mix(np.array([1.0]), T)[0]) for s in sp8])
        am, _, _, _ = mech8_k0.mix(X, T)
        assert am == pytest.approx(float(X @ sq) ** 2, rel=1e-13)


def test_permutation_invariance(orc, sp8):
    kij = synth.synthetic_kij(8)
    perm = np.random.default_rng(5).permutation(8)
    m1 = orc.Mech(sp8, kij)
    m2 = orc.Mech([sp8[i] for i in perm], kij[np.ix_(perm, perm)])
    P, T, Y = synth.flame_field(8, seed=2)
    a = m1.state_PT(P, T, Y)
    b = m2.state_PT(P, T, Y[perm])
    for f in ("Z", "rho", "h", "cp", "c", "mu", "lambda"):
        np.testing.assert_allclose(a[f], b[f], rtol=1e-12, err_msg=f)


@pytest.mark.parametrize("name", ["O2", "H2O"])
def test_identical_species_mixture_is_the_pure_fluid(orc, name):
    """Two copies of one species at any split must give the pure fluid (PR and both Chung
    mixtures); H2O carries a dipole and an association factor."""
    s = synth.load_species([name])[0]
    m2 = orc.Mech([s, dict(s)])
    m1 = orc.Mech([s])
    P = np.array([10e6, 1e5, 20e6])
    T = np.array([700.0, 1500.0, 2900.0])
    for y in (0.1, 0.5, 0.93):
        a = m2.state_PT(P, T, np.array([[y] * 3, [1 - y] * 3]))
        b = m1.state_PT(P, T, np.ones((1, 3)))
        for f in ("Z", "rho", "h", "cp", "c", "mu", "lambda"):
            np.testing.assert_allclose(a[f], b[f], rtol=1e-12, err_msg=f)


# ---------------------------------------------------------------------------------------
# Temperature inversion
# ---------------------------------------------------------------------------------------

def test_rhoe_round_trip(orc, mech8):
    P, T, Y = synth.flame_field(16, seed=4)
    a = mech8.state_PT(P, T, Y, transport=False)
    b = mech8.state_rhoe(a["rho"], a["e"], Y, transport=False)
    tol = 1e-12 * np.maximum(1.0, a["kappa_T"]) * 4
    assert np.all(np.abs(b["T"] / T - 1) <= tol)
    assert np.all(np.abs(b["P"] / P - 1) < 1e-9)


def test_rhoe_bracket_and_nonphysical_flags(orc, mech8):
    Y = np.zeros((8, 6))
    Y[1] = 1.0
    rho = np.array([100.0, 100.0, -1.0, 100.0, 100.0, 100.0])
    e = np.array([5e7, -5e7, 0.0, 0.0, np.nan, 0.0])
    Y[:, 5] = 0.0
    Y[1, 5] = 0.9  # sum of Y is 0.9
    r = mech8.state_rhoe(rho, e, Y, transport=False)
    assert r["status"][0] & orc.BRACKET and r["status"][1] & orc.BRACKET
    assert r["status"][2] & orc.NONPHYS and r["status"][4] & orc.NONPHYS
    assert r["status"][5] & orc.NONPHYS
    assert r["status"][3] == 0 and np.isfinite(r["T"][3])
    assert np.all(np.isnan(r["T"][[0, 1, 2, 4, 5]]))


# ---------------------------------------------------------------------------------------
# Chung transport (Section 2; Table 1 is the paper's only printed property value)
# ---------------------------------------------------------------------------------------

def test_table1_kinematic_viscosity_pr_density(orc):
    """nu = mu/rho of O2 at 150 K, 10 MPa with PR density. Soft pin (2 %): the value also
    depends on species constants the paper does not print."""
    g = gold("paper_values.json")
    s = synth.load_species(["O2"])
    r = orc.Mech(s).state_PT([g["state_O2"]["P"]], [g["state_O2"]["T"]], [[1.0]])
    nu = r["mu"][0] / r["rho"][0]
    assert abs(nu / g["nu_min_real_gas"]["value"] - 1) < 0.02
    # the Reynolds numbers of Table 1 follow from u0 L0 / nu
    assert abs(g["u0"]["value"] * g["L0"]["value"] / g["nu_min_real_gas"]["value"] - g["Re_real_gas"]["value"]) < 1


def test_table1_kinematic_viscosity_ideal_density(orc):
    g = gold("paper_values.json")
    s = synth.load_species(["O2"])
    T, P = g["state_O2"]["T"], g["state_O2"]["P"]
    rho = P * s[0]["W"] / (R * T)
    r = orc.Mech(s).state_vT([s[0]["W"] / rho], [T], [[1.0]])
    nu = r["mu"][0] / rho
    assert abs(nu / g["nu_min_ideal_gas"]["value"] - 1) < 0.02
    # the paper truncates: u0 L0 / nu = 1821.8 is printed as 1821
    assert abs(g["u0"]["value"] * g["L0"]["value"] / g["nu_min_ideal_gas"]["value"] - g["Re_ideal_gas"]["value"]) < 1
    assert g["L0"]["value"] / g["u0"]["value"] == pytest.approx(g["tau_ref"]["value"])


def test_neufeld_collision_integral_against_lj_table(orc):
    tab = gold("textbook_values.json")["lj_omega22"]
    for k, v in tab.items():
        if k.startswith("_"):
            continue
        assert abs(orc.omega_v(float(k)) / v - 1) < 0.005


def test_chung_dense_viscosity_dilute_limit(orc):
    """y -> 0 of the dense formula equals the low-pressure Chung viscosity; the two
    published prefactors agree to their printed digits (36.344 sqrt(1.2593) = 40.7847
    vs 40.785), hence 2e-5."""
    for (Tc, Vc, M, w, mr, k) in [(154.58, 73.4, 31.998, 0.0222, 0, 0), (647.14, 55.95, 18.015, 0.344, 1.24, 0.076)]:
        for T in (200.0, 1000.0, 3000.0):
            a = orc.chung_mu(T, 1e-9, Tc, Vc, M, w, mr, k)
            b = orc.chung_mu0(T, Tc, Vc, M, w, mr, k)
            assert a == pytest.approx(b, rel=2e-5)


def test_chung_conductivity_monatomic_dilute_limit(orc):
    """For Cv = 3/2 R (alpha = 0, Psi = 1) the dilute Chung conductivity is the
    Chapman-Enskog monatomic result lambda = (15/4) (R/M) mu (31.2 vs 3.75 R = 31.18)."""
    Tc, Vc, M, w = 150.86, 74.57, 39.948, -0.002
    for T in (300.0, 1000.0):
        lam = orc.chung_lambda(T, 1e-9, Tc, Vc, M, w, 0.0, 0.0, 1.5 * R)
        mu = orc.chung_mu0(T, Tc, Vc, M, w, 0.0, 0.0)
        assert lam == pytest.approx(3.75 * R * mu / (M * 1e-3), rel=1e-3)


def test_transport_positive_on_flame_field(mech8):
    P, T, Y = synth.flame_field(12, seed=9)
    r = mech8.state_PT(P, T, Y)
    assert np.all(r["mu"] > 0) and np.all(r["lambda"] > 0)
    assert np.all((r["mu"] > 1e-6) & (r["mu"] < 1e-3))
    assert np.all((r["lambda"] > 1e-3) & (r["lambda"] < 2.0))


def test_single_species_mechanism_is_textbook_chung(orc):
    """For a pure fluid the mixture model reduces to Chung's textbook dense viscosity and
    conductivity (up to the printed rounding of 40.785 = 36.344 sqrt(1.2593))."""
    for name in ("O2", "CH4", "H2O", "CO2"):
        s = synth.load_species([name])[0]
        P = np.array([10e6, 2e6, 10e6])
        T = np.array([s["Tc"] * 0.97, 900.0, 2500.0])
        r = orc.Mech([s]).state_PT(P, T, np.ones((1, 3)))
        for k in range(3):
            rho_m = r["rho"][k] / s["W"]
            args = (s["Tc"], s["Vc"] * 1e6, s["W"] * 1e3, s["omega"], 0.0, s["kappa"])
            mu = orc.chung_mu(T[k], rho_m, *args)
            lam = orc.chung_lambda(T[k], rho_m, *args, r["cv_ig"][k] * s["W"])
            assert r["mu"][k] == pytest.approx(mu, rel=2e-5)
            assert r["lambda"][k] == pytest.approx(lam, rel=2e-5)


def test_polar_pseudo_mixture_is_singular_hence_nonpolar_data(orc):
    """Why the species file uses dipole = 0: with the physical 1.8 D of H2O, Chung's
    pseudo-mixture viscosity of a CH4/H2O gas changes sign as the H2O fraction grows
    (the denominator of G2 crosses zero); with the non-polar treatment it stays positive."""
    sp = synth.load_species(["CH4", "H2O"])
    polar = [dict(sp[0]), dict(sp[1], dipole=sp[1]["dipole_physical"])]
    y = np.linspace(0.01, 0.6, 300)
    Y = np.stack([1 - y, y])
    P = np.full(y.size, 20e6)
    T = np.full(y.size, 1100.0)
    mu_polar = orc.Mech(polar).state_PT(P, T, Y)["mu"]
    mu_np = orc.Mech(sp).state_PT(P, T, Y)["mu"]
    assert np.any(mu_polar < 0)
    assert np.all((mu_np > 1e-6) & (mu_np < 1e-3))


def test_energy_equation_of_state(orc):
    """(de/dv)_T = T (dP/dT)_v - P (the thermodynamic equation of state): pins the
    departure energy against Eq. (1) itself, both sides by finite differences."""
    sp, P, T, Y = _fd_states()
    m = orc.Mech(sp, [[0, 0.03], [0.03, 0]])
    v = m.state_PT(P, T, Y, transport=False)["v"]
    dv, dT = 1e-6 * v, 1e-6 * T
    ep = m.state_vT(v + dv, T, Y, transport=False)
    em = m.state_vT(v - dv, T, Y, transport=False)
    W = ep["W"]
    dedv = (ep["e"] - em["e"]) * W / (2 * dv)            # molar e per molar v
    Pp = m.state_vT(v, T + dT, Y, transport=False)["P"]
    Pm = m.state_vT(v, T - dT, Y, transport=False)["P"]
    P0 = m.state_vT(v, T, Y, transport=False)["P"]
    rhs = T * (Pp - Pm) / (2 * dT) - P0
    scale = np.abs(T * (Pp - Pm) / (2 * dT)) + np.abs(P0)
    assert np.max(np.abs(dedv - rhs) / scale) < 1e-5


def test_chung_viscosity_has_a_pole_at_negative_pseudo_acentric_factor(orc):
    """A property of the method: with H2 (omega = -0.216) the pseudo-mixture acentric factor
    of H2/CH4 sweeps through -0.0674, where Chung's E1 E4 + E2 + E3 vanishes and the dense
    viscosity has a pole (changes sign); flame-like H2 fractions stay far from it."""
    sp = synth.load_species(["CH4", "H2"])
    xh2 = np.linspace(0.02, 0.98, 400)
    W = np.array([s["W"] for s in sp])
    Y = np.stack([(1 - xh2) * W[0], xh2 * W[1]])
    Y /= Y.sum(0, keepdims=True)
    r = orc.Mech(sp).state_PT(np.full(400, 10e6), np.full(400, 600.0), Y)
    assert np.any(r["mu"] < 0) and np.any(r["mu"] > 0)
    lean = xh2 < 0.05
    assert np.all(r["mu"][lean] > 0)
