"""GPU parity of the (h, P, Y) mode and of the solver outputs psi, alpha and h_i/(R T).

The pressure-based solver hands the property package enthalpy and pressure each
pressure-correction loop (Section 3) and its surrogate targets include psi = d rho/d p at
constant enthalpy, the thermal diffusivity and the species' h_i/(R T) (Section 4.1).  Every
expected value comes from the CPU oracle on seeded synthetic inputs.

Tolerances.  FP64 outputs at a given (P, T) carry relative rounding errors bounded by
1e-12 times the cell condition number of the (P, T, Y) state (parity_util.cell_kappa).  In
(h, P, Y) mode T itself is only defined to h's rounding, a relative uncertainty of
kappa_hT = h_scale/(T cp) ulps, which each output inherits through its temperature
sensitivity |T d ln(out)/dT|_P; that sensitivity is taken from oracle central differences.
"""
import numpy as np
import pytest

import synth
from parity_util import FIELDS, cell_kappa, compare, rel_err_stats, run_gpu

pytestmark = pytest.mark.gpu

FP64_RTOL = 1e-12
# Mixed precision on the flame field: relative 2e-5 (measured at most 3.4e-6, mu)
MIXED_RTOL = 2e-5
SOLVER = ("psi", "alpha")
ALL = FIELDS + SOLVER


@pytest.fixture(scope="module")
def props():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_04830_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def sp8():
    return synth.load_species(synth.FLAME_SPECIES)


@pytest.fixture(scope="module")
def kij8():
    return synth.synthetic_kij(8)


def _scale(ref, f):
    if f == "h":
        return ref["h_scale"]
    if f == "e":
        return ref["e_scale"]
    return np.abs(ref[f])


def hp_compare(om, g, ref, P, Y, rtol, fields=ALL):
    """worst err/tol per output for (h, P, Y) results (see the module docstring)."""
    T = ref["T"]
    d = 1e-6
    up = om.state_PT(P, T * (1 + d), Y)
    dn = om.state_PT(P, T * (1 - d), Y)
    k_hT = ref["h_scale"] / (T * np.abs(ref["cp"]))
    base = cell_kappa(ref, 0)
    worst = {}
    for f in fields:
        if f == "T":
            sens = np.ones_like(T)
        else:
            sens = np.abs(up[f] - dn[f]) / (2 * d) / _scale(ref, f)
        tol = rtol * (base + 4.0 * k_hT * sens) * _scale(ref, f)
        err = np.abs(g[f] - ref[f])
        both_nan = np.isnan(g[f]) & np.isnan(ref[f])
        err = np.where(both_nan, 0.0, np.where(np.isnan(err), np.inf, err))
        worst[f] = float(np.max(err / np.maximum(tol, 1e-300)))
    return worst


def hrt_compare(sp, g, ref, T_rel_unc, rtol):
    """h_i/(R T) crosses zero (formation enthalpies of either sign), so each species is
    compared against the magnitudes it is summed from, |sensible part| + |a6|/T, plus
    the effect of T's own uncertainty, (c_p,i/R + |h_i/RT|) dT/T with c_p,i/R < 20."""
    ns = len(sp)
    T = ref["T"]
    worst = 0.0
    for i, s in enumerate(sp):
        a6 = np.where(T < s["Tmid"], s["nasa_lo"][5], s["nasa_hi"][5])
        r = ref["hRT"][:, i]
        mag = np.abs(r - a6 / T) + np.abs(a6 / T)
        tol = rtol * (4.0 * mag + 1.0) + T_rel_unc * (20.0 + np.abs(r))
        err = np.abs(g["hRT"][i] - r)
        ok = np.isfinite(r)
        assert np.array_equal(np.isnan(g["hRT"][i]), np.isnan(r))
        if ok.any():
            worst = max(worst, float(np.max(err[ok] / tol[ok])))
    assert ns == g["hRT"].shape[0]
    return worst


def _report(name, worst):
    print(f"\n[{name}] worst err/tol: " + ", ".join(f"{k}={v:.3g}" for k, v in worst.items()), flush=True)


# ------------------------------------------------------------------ (h, P, Y) on the flame field

@pytest.mark.parametrize("guess", [True, False])
def test_hpy_fp64_flame_field(props, orc, sp8, kij8, guess):
    P, T, Y = synth.flame_field(23, seed=1)          # 12167 cells: ragged tail
    n = T.size
    om = orc.Mech(sp8, kij8)
    h = om.state_PT(P, T, Y, transport=False)["h"]
    ref = om.state_hP(h, P, Y)
    Tg = synth.temperature_guess(T) if guess else None
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.HPY, props.FP64, n,
                {"h": h, "P": P, "Y": Y, "T_guess": Tg}, fields=ALL + ("hRT", "iters"), ns=8)
    worst = hp_compare(om, g, ref, P, Y, FP64_RTOL)
    k_hT = ref["h_scale"] / (T * np.abs(ref["cp"]))
    worst["hRT"] = hrt_compare(sp8, g, ref, FP64_RTOL * 4 * k_hT, FP64_RTOL)
    _report(f"hpy fp64 guess={guess}", worst)
    assert max(worst.values()) <= 1.0, worst
    assert np.array_equal(g["status"], ref["status"])
    assert np.max(np.abs(g["T"] / T - 1)) < 1e-11
    print(f"[hpy fp64 guess={guess}] evaluations: mean {g['iters'].mean():.2f}, max {g['iters'].max()}")
    assert g["iters"].max() <= (8 if guess else 40)


def test_hpy_fp64_two_species_cells(props, orc):
    """Independent CH4/O2 cells at 5-15 MPa and 100-1000 K (liquid-like to gas-like)."""
    sp = synth.load_species(["CH4", "O2"])
    kij = [[0.0, 0.03], [0.03, 0.0]]
    P, T, Y = synth.cells_uniform(4096, seed=0)
    om = orc.Mech(sp, kij)
    h = om.state_PT(P, T, Y, transport=False)["h"]
    ref = om.state_hP(h, P, Y)
    g = run_gpu(props, props.Mechanism(sp, kij), props.HPY, props.FP64, T.size, {"h": h, "P": P, "Y": Y},
                fields=ALL)
    worst = hp_compare(om, g, ref, P, Y, FP64_RTOL)
    _report("hpy fp64 two species", worst)
    assert max(worst.values()) <= 1.0, worst
    assert np.array_equal(g["status"], ref["status"])


def test_hpy_full_field_sampled(props, orc, sp8, kij8):
    """The 128^3 flame field in the benchmark's launch configuration; a seeded sample of
    cells is recomputed by the oracle one by one."""
    import torch
    P, T, Y = synth.flame_field(128, seed=1)
    n = T.size
    om = orc.Mech(sp8, kij8)
    idx = np.random.default_rng(321).choice(n, 2000, replace=False)
    idx = np.concatenate([idx, [0, n - 1]])
    # the solver state of every cell (the oracle's (P, T, Y) enthalpy, without transport)
    h = om.state_PT(P, T, Y, transport=False)["h"]
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.HPY, props.FP64, n,
                {"h": h, "P": P, "Y": Y, "T_guess": synth.temperature_guess(T)}, fields=ALL)
    Ys = np.ascontiguousarray(Y[:, idx])
    ref = om.state_hP(h[idx], P[idx], Ys)
    gs = {k: v[idx] for k, v in g.items()}
    worst = hp_compare(om, gs, ref, P[idx], Ys, FP64_RTOL)
    _report("hpy fp64 128^3 sampled", worst)
    assert max(worst.values()) <= 1.0, worst
    assert np.all(g["status"] == 0)
    assert np.max(np.abs(g["T"] / T - 1)) < 1e-10
    assert np.all(g["psi"] > 0) and np.all(g["alpha"] > 0)
    del g
    torch.cuda.empty_cache()


def test_hpy_flags(props, orc, sp8, kij8):
    n = 8
    Y = np.zeros((8, n))
    Y[1] = 1.0
    P = np.array([10e6, 10e6, -1.0, 10e6, 10e6, 10e6, 10e6, np.nan])
    h = np.array([5e7, -5e7, 0.0, 0.0, np.nan, 0.0, 1e5, 0.0])
    Y[:, 5] = 0.0
    Y[1, 5] = 0.9          # sum Y != 1
    Y[:, 6] = 0.0
    Y[0, 6], Y[1, 6] = -0.5, 1.5   # negative mass fraction
    ref = orc.Mech(sp8, kij8).state_hP(h, P, Y)
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.HPY, props.FP64, n, {"h": h, "P": P, "Y": Y},
                fields=ALL + ("hRT",), ns=8)
    assert np.array_equal(g["status"], ref["status"]), (g["status"], ref["status"])
    for f in ALL:
        assert np.array_equal(np.isnan(g[f]), np.isnan(ref[f])), f
    assert np.array_equal(np.isnan(g["hRT"]), np.isnan(ref["hRT"][:, :8].T))


def test_hpy_in_the_enthalpy_gap(props, orc):
    """Pure O2 at 3 MPa: an h* inside the jump of h(T) at the liquid/vapour root switch
    has no root; both sides end at the switch temperature."""
    sp = synth.load_species(["O2"])
    om = orc.Mech(sp)
    P = 3.0e6
    T = np.linspace(100.0, 150.0, 501)
    s = om.state_PT(np.full(T.size, P), T, np.ones((1, T.size)), transport=False)
    k = int(np.argmax(np.diff(s["Z"])))
    hl, hv = s["h"][k], s["h"][k + 1]
    h = np.array([hl - 1e4, 0.5 * (hl + hv), hv + 1e4])
    Pv = np.full(3, P)
    ref = om.state_hP(h, Pv, np.ones((1, 3)), transport=False)
    g = run_gpu(props, props.Mechanism(sp), props.HPY, props.FP64, 3, {"h": h, "P": Pv, "Y": np.ones((1, 3))},
                fields=("T", "Z", "rho"))
    assert np.abs(g["T"][1] / ref["T"][1] - 1) < 1e-9
    for j in (0, 2):
        assert np.abs(g["T"][j] / ref["T"][j] - 1) < 1e-11
        assert np.abs(g["rho"][j] / ref["rho"][j] - 1) < 1e-9


# ------------------------------------------------------------------ solver outputs in every mode

def test_solver_outputs_pty_and_rhoey(props, orc, sp8, kij8):
    P, T, Y = synth.flame_field(16, seed=7)
    n = T.size
    om = orc.Mech(sp8, kij8)
    m = props.Mechanism(sp8, kij8)
    ref = om.state_PT(P, T, Y)
    g = run_gpu(props, m, props.PTY, props.FP64, n, {"P": P, "T": T, "Y": Y}, fields=ALL + ("hRT",), ns=8)
    worst = compare(g, ref, 0, FP64_RTOL, fields=ALL)
    worst["hRT"] = hrt_compare(sp8, g, ref, 0.0, FP64_RTOL)
    _report("pty fp64 solver outputs", worst)
    assert max(worst.values()) <= 1.0, worst
    refr = om.state_rhoe(ref["rho"], ref["e"], Y)
    g = run_gpu(props, m, props.RHOEY, props.FP64, n, {"rho": ref["rho"], "e": ref["e"], "Y": Y},
                fields=ALL + ("hRT",), ns=8)
    worst = compare(g, refr, 1, FP64_RTOL, fields=ALL)
    worst["hRT"] = hrt_compare(sp8, g, refr, FP64_RTOL * cell_kappa(refr, 1), FP64_RTOL)
    _report("rhoey fp64 solver outputs", worst)
    assert max(worst.values()) <= 1.0, worst


def test_alpha_alone_runs_transport(props, orc, sp8, kij8):
    """alpha requested without mu and lambda still evaluates the transport model."""
    P, T, Y = synth.flame_field(6, seed=3)
    ref = orc.Mech(sp8, kij8).state_PT(P, T, Y)
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.PTY, props.FP64, T.size, {"P": P, "T": T, "Y": Y},
                fields=("alpha",))
    worst = compare(g, ref, 0, FP64_RTOL, fields=("alpha",))
    assert worst["alpha"] <= 1.0, worst


@pytest.mark.parametrize("ns", [1, 2, 5])
def test_hpy_species_counts(props, orc, sp8, ns):
    sp = sp8[:ns]
    rng = np.random.default_rng(40 + ns)
    n = 777
    Y = rng.dirichlet(np.ones(ns), n).T.copy()
    P = rng.uniform(5e6, 2e7, n)
    T = rng.uniform(250.0, 2500.0, n)
    kij = synth.synthetic_kij(ns, seed=ns)
    om = orc.Mech(sp, kij)
    h = om.state_PT(P, T, Y, transport=False)["h"]
    ref = om.state_hP(h, P, Y)
    g = run_gpu(props, props.Mechanism(sp, kij), props.HPY, props.FP64, n, {"h": h, "P": P, "Y": Y},
                fields=ALL + ("hRT",), ns=ns)
    worst = hp_compare(om, g, ref, P, Y, FP64_RTOL)
    k_hT = ref["h_scale"] / (ref["T"] * np.abs(ref["cp"]))
    worst["hRT"] = hrt_compare(sp, g, ref, FP64_RTOL * 4 * k_hT, FP64_RTOL)
    assert max(worst.values()) <= 1.0, worst


# ------------------------------------------------------------------ mixed precision

def test_hpy_mixed_error_report(props, orc, sp8, kij8):
    P, T, Y = synth.flame_field(24, seed=1)
    n = T.size
    om = orc.Mech(sp8, kij8)
    h = om.state_PT(P, T, Y, transport=False)["h"]
    ref = om.state_hP(h, P, Y)
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.HPY, props.MIXED, n,
                {"h": h, "P": P, "Y": Y, "T_guess": synth.temperature_guess(T)}, fields=ALL + ("iters",))
    assert np.all(g["status"] == 0), np.unique(g["status"])
    assert g["iters"].max() <= 8, np.bincount(g["iters"].astype(np.int64))
    stats = rel_err_stats(g, ref, fields=ALL)
    print("\n[mixed hpy] max/rms rel err: " + ", ".join(f"{k}={v[0]:.2e}/{v[1]:.2e}" for k, v in stats.items()))
    for f in ALL:
        assert stats[f][0] <= MIXED_RTOL, (f, stats[f])


@pytest.mark.parametrize("guess_rel", [0.3, None])
def test_hpy_fp64_wide_states_poor_guess(props, orc, sp8, kij8, guess_rel):
    """(h, P, Y) on states far from the flame field's (T ~ U[100, 4800] K, P ~ U[1, 30] MPa,
    random 8-species compositions) from a poor guess or from the bracket top: the Newton
    iteration with its bisection fallbacks and its look-ahead stop (three steps of consistent
    quadratic contraction) meets the oracle at every cell.  Thermodynamic outputs only: at
    such compositions Chung's viscosity cancels (see the (rho, e, Y) wide-state test)."""
    rng = np.random.default_rng(79)
    n = 2048
    P = rng.uniform(1.0e6, 30.0e6, n)
    T = rng.uniform(100.0, 4800.0, n)
    Y = rng.uniform(0.0, 1.0, (8, n))
    Y /= Y.sum(axis=0)
    om = orc.Mech(sp8, kij8)
    h = om.state_PT(P, T, Y, transport=False)["h"]
    ref = om.state_hP(h, P, Y)
    Tg = None if guess_rel is None else synth.temperature_guess(T, seed=80, rel=guess_rel)
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.HPY, props.FP64, n,
                {"h": h, "P": P, "Y": Y, "T_guess": Tg}, fields=FIELDS + ("iters",))
    assert np.array_equal(g["status"], ref["status"]), np.unique(g["status"] - ref["status"])
    worst = hp_compare(om, g, ref, P, Y, FP64_RTOL, fields=[f for f in FIELDS if f not in ("mu", "lambda")])
    print(f"\n[hpy fp64 wide states guess={guess_rel}] worst err/tol: "
          + ", ".join(f"{k}={v:.3g}" for k, v in worst.items()), flush=True)
    assert max(worst.values()) <= 1.0, worst
    assert g["iters"].max() <= 40, np.bincount(g["iters"].astype(np.int64))


def test_hpy_newton_iteration_limit_and_empty_launch(props, orc, sp8, kij8):
    import torch
    P, T, Y = synth.flame_field(6, seed=3)
    h = orc.Mech(sp8, kij8).state_PT(P, T, Y, transport=False)["h"]
    m = props.Mechanism(sp8, kij8)
    m.set_newton(max_iter=1)
    g = run_gpu(props, m, props.HPY, props.FP64, T.size, {"h": h, "P": P, "Y": Y}, fields=("T",))
    assert np.all(g["status"] & 2)
    m.set_newton(100, 1e-10)
    g = run_gpu(props, m, props.HPY, props.FP64, T.size, {"h": h, "P": P, "Y": Y}, fields=("T",))
    assert np.all(g["status"] == 0)
    z = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    props.pr(m, props.HPY, props.FP64, {"h": z, "P": z, "Y": z}, {"T": z}, 0)
    with pytest.raises(props.PropsError):
        props.pr(m, props.HPY, props.FP64, {"P": z, "Y": z}, {"T": z}, 1)    # h missing


def test_hpy_deterministic_bitwise(props, orc, sp8, kij8):
    P, T, Y = synth.flame_field(12, seed=5)
    h = orc.Mech(sp8, kij8).state_PT(P, T, Y, transport=False)["h"]
    m = props.Mechanism(sp8, kij8)
    inp = {"h": h, "P": P, "Y": Y, "T_guess": synth.temperature_guess(T)}
    a = run_gpu(props, m, props.HPY, props.FP64, T.size, inp, fields=ALL + ("hRT",), ns=8)
    b = run_gpu(props, m, props.HPY, props.FP64, T.size, inp, fields=ALL + ("hRT",), ns=8)
    for f in ALL + ("hRT",):
        assert np.array_equal(a[f].view(np.int64), b[f].view(np.int64)), f
