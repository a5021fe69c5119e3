"""GPU parity of the Peng-Robinson property path (props_pr) against the CPU oracle.

Every input is seeded and synthetic (synth), every expected value comes from the oracle.
FP64 bar: relative 1e-12 scaled by each cell's condition number (cell_kappa).
"""
import numpy as np
import pytest

import synth
from parity_util import FIELDS, chung_kappa, compare, rel_err_stats, run_gpu

pytestmark = pytest.mark.gpu

FP64_RTOL = 1e-12
# Mixed precision (FP32 where the policy allows): relative 2e-5 on the flame field, about 3x
# the largest error measured there (6.7e-6, P from (rho, e)); on wide states 1e-6 times the
# cell's condition number, since the FP32 parts round at 6e-8 relative before the same
# cancellations the FP64 bar scales with (measured worst 0.17 of that bar, c).
MIXED_RTOL = 2e-5
MIXED_KAPPA_RTOL = 1e-6


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


def _report(name, worst):
    print(f"\n[{name}] worst err/tol: " + ", ".join(f"{k}={v:.3g}" for k, v in worst.items()), flush=True)


# ------------------------------------------------------------------ (P, T, Y), 2 species

@pytest.mark.parametrize("n", [4096, 4095, 1, 257])
def test_pty_fp64_two_species_uniform_cells(props, orc, n):
    sp = synth.load_species(["CH4", "O2"])
    P, T, Y = synth.cells_uniform(4096, seed=0)
    P, T, Y = P[:n], T[:n], np.ascontiguousarray(Y[:, :n])
    om = orc.Mech(sp)
    ref = om.state_PT(P, T, Y)
    gm = props.Mechanism(sp)
    g = run_gpu(props, gm, props.PTY, props.FP64, n, {"P": P, "T": T, "Y": Y})
    worst = compare(g, ref, 0, FP64_RTOL)
    _report(f"pty fp64 n={n}", worst)
    assert max(worst.values()) <= 1.0, worst
    assert np.array_equal(g["status"], ref["status"])


def test_pty_fp64_kij_two_species(props, orc):
    sp = synth.load_species(["CH4", "O2"])
    kij = [[0.0, 0.05], [0.05, 0.0]]
    P, T, Y = synth.cells_uniform(4096, seed=10)
    ref = orc.Mech(sp, kij).state_PT(P, T, Y)
    g = run_gpu(props, props.Mechanism(sp, kij), props.PTY, props.FP64, 4096, {"P": P, "T": T, "Y": Y})
    worst = compare(g, ref, 0, FP64_RTOL)
    _report("pty fp64 kij", worst)
    assert max(worst.values()) <= 1.0, worst


# ------------------------------------------------------------------ (P, T, Y), 8 species flame field

def test_pty_fp64_flame_field(props, orc, sp8, kij8):
    P, T, Y = synth.flame_field(23, seed=1)      # 12167 cells: ragged tail
    n = T.size
    ref = orc.Mech(sp8, kij8).state_PT(P, T, Y)
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.PTY, props.FP64, n, {"P": P, "T": T, "Y": Y})
    worst = compare(g, ref, 0, FP64_RTOL)
    _report("pty fp64 flame", worst)
    assert max(worst.values()) <= 1.0, worst
    assert np.array_equal(g["status"], ref["status"])


# ------------------------------------------------------------------ (rho, e, Y) Newton

@pytest.mark.parametrize("guess", [True, False])
def test_rhoey_fp64_flame_field(props, orc, sp8, kij8, guess):
    P, T, Y = synth.flame_field(23, seed=1)
    n = T.size
    om = orc.Mech(sp8, kij8)
    st = om.state_PT(P, T, Y, transport=False)
    rho, e = st["rho"], st["e"]
    ref = om.state_rhoe(rho, e, Y)
    Tg = synth.temperature_guess(T) if guess else None
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.RHOEY, props.FP64, n,
                {"rho": rho, "e": e, "Y": Y, "T_guess": Tg})
    worst = compare(g, ref, 1, FP64_RTOL)
    _report(f"rhoey fp64 guess={guess}", worst)
    assert max(worst.values()) <= 1.0, worst
    assert np.array_equal(g["status"], ref["status"])
    assert np.max(np.abs(g["T"] / T - 1)) < 1e-11


@pytest.mark.parametrize("guess_rel", [0.3, None])
def test_rhoey_fp64_wide_states_poor_guess(props, orc, sp8, kij8, guess_rel):
    """(rho, e, Y) on states far from the flame field's: T ~ U[100, 4800] K (across the NASA
    range switch and every sign change of the mixing sum), P ~ U[1, 30] MPa, random
    8-species compositions, started from a poor guess (30 % spread, clipped into the bracket
    by the kernel where it falls outside) or from the top of the bracket: the iteration's
    bisection fallbacks and third-order steps meet the oracle's plain Newton at every cell.
    The thermodynamic outputs are compared here, transport in the test below."""
    rng = np.random.default_rng(77)
    n = 2048
    P = rng.uniform(1.0e6, 30.0e6, n)
    T = rng.uniform(100.0, 4800.0, n)
    Y = rng.uniform(0.0, 1.0, (8, n))
    Y /= Y.sum(axis=0)
    om = orc.Mech(sp8, kij8)
    st = om.state_PT(P, T, Y, transport=False)
    ref = om.state_rhoe(st["rho"], st["e"], Y)
    Tg = None if guess_rel is None else synth.temperature_guess(T, seed=78, rel=guess_rel)
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.RHOEY, props.FP64, n,
                {"rho": st["rho"], "e": st["e"], "Y": Y, "T_guess": Tg}, fields=FIELDS + ("iters",))
    assert np.array_equal(g["status"], ref["status"]), np.unique(g["status"] - ref["status"])
    worst = compare(g, ref, 1, FP64_RTOL, fields=[f for f in FIELDS if f not in ("mu", "lambda")])
    _report(f"rhoey fp64 wide states guess={guess_rel}", worst)
    assert max(worst.values()) <= 1.0, worst
    assert g["iters"].max() <= 40, np.bincount(g["iters"].astype(np.int64))


def test_rhoey_fp64_wide_states_transport(props, orc, sp8, kij8):
    """Chung's mu and lambda on the wide states above.  At such arbitrary compositions and
    densities the dense-fluid terms can cancel against the dilute ones (mu turns negative on
    about 1 % of the cells, R30), and for mixtures rich in H2 the G2 denominator nears zero
    (R31), so each cell's bar is 1e-12 relative to the sum of the magnitudes of the output's
    terms (the oracle's mu_scale, lambda_scale), times the thermodynamic condition number
    (T and rho enter the correlation) and the G2 denominator's (chung_kappa)."""
    rng = np.random.default_rng(77)
    n = 2048
    P = rng.uniform(1.0e6, 30.0e6, n)
    T = rng.uniform(100.0, 4800.0, n)
    Y = rng.uniform(0.0, 1.0, (8, n))
    Y /= Y.sum(axis=0)
    om = orc.Mech(sp8, kij8)
    st = om.state_PT(P, T, Y, transport=False)
    ref = om.state_rhoe(st["rho"], st["e"], Y)
    Tg = synth.temperature_guess(T, seed=78, rel=0.3)
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.RHOEY, props.FP64, n,
                {"rho": st["rho"], "e": st["e"], "Y": Y, "T_guess": Tg})
    assert np.array_equal(g["status"], ref["status"])
    kmu, klam = chung_kappa(sp8, Y)
    ok = ref["status"] == 0
    print(f"\n[wide transport] mu < 0 on {int((ref['mu'][ok] < 0).sum())} of {int(ok.sum())} cells; "
          f"max cancellation {np.nanmax(ref['mu_scale'][ok] / np.abs(ref['mu'][ok])):.3g} (mu), "
          f"{np.nanmax(ref['lambda_scale'][ok] / np.abs(ref['lambda'][ok])):.3g} (lambda); max G2 kappa "
          f"{kmu.max():.3g} / {klam.max():.3g}", flush=True)
    worst = compare(g, ref, 1, FP64_RTOL, fields=("mu", "lambda"), mask=ok, extra={"mu": kmu, "lambda": klam},
                    scales={"mu": ref["mu_scale"], "lambda": ref["lambda_scale"]})
    _report("rhoey fp64 wide states transport", worst)
    assert max(worst.values()) <= 1.0, worst


@pytest.mark.parametrize("mode", ["RHOEY", "HPY"])
def test_mixed_precision_wide_states_poor_guess(props, orc, sp8, kij8, mode):
    """The mixed-precision inversions on the wide states of the FP64 test above, from a poor
    guess: every cell converges, thermodynamic outputs within the mixed-precision bar."""
    rng = np.random.default_rng(77)
    n = 2048
    P = rng.uniform(1.0e6, 30.0e6, n)
    T = rng.uniform(100.0, 4800.0, n)
    Y = rng.uniform(0.0, 1.0, (8, n))
    Y /= Y.sum(axis=0)
    om = orc.Mech(sp8, kij8)
    st = om.state_PT(P, T, Y, transport=False)
    Tg = synth.temperature_guess(T, seed=78, rel=0.3)
    if mode == "RHOEY":
        ref = om.state_rhoe(st["rho"], st["e"], Y)
        inputs = {"rho": st["rho"], "e": st["e"], "Y": Y, "T_guess": Tg}
    else:
        ref = om.state_hP(st["h"], P, Y)
        inputs = {"h": st["h"], "P": P, "Y": Y, "T_guess": Tg}
    g = run_gpu(props, props.Mechanism(sp8, kij8), getattr(props, mode), props.MIXED, n, inputs,
                fields=FIELDS + ("iters",))
    assert np.array_equal(g["status"], ref["status"]), np.unique(g["status"] - ref["status"])
    fields = [f for f in FIELDS if f not in ("mu", "lambda")]
    stats = rel_err_stats(g, ref, fields=fields)
    print(f"\n[mixed {mode.lower()} wide states] max/rms rel err: "
          + ", ".join(f"{k}={v[0]:.2e}/{v[1]:.2e}" for k, v in stats.items()), flush=True)
    worst = compare(g, ref, 1, MIXED_KAPPA_RTOL, fields=fields)
    _report(f"mixed {mode.lower()} wide states (1e-6 x kappa)", worst)
    assert max(worst.values()) <= 1.0, worst
    assert g["iters"].max() <= 40, np.bincount(g["iters"].astype(np.int64))


def test_rhoey_fp64_full_field_sampled(props, orc, sp8, kij8):
    """The 128^3 flame field in the benchmark's launch configuration; a seeded sample of
    cells is recomputed by the oracle one by one."""
    import torch
    P, T, Y = synth.flame_field(128, seed=1)
    n = T.size
    om = orc.Mech(sp8, kij8)
    st = om.state_PT(P, T, Y, transport=False)
    Tg = synth.temperature_guess(T)
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.RHOEY, props.FP64, n,
                {"rho": st["rho"], "e": st["e"], "Y": Y, "T_guess": Tg})
    idx = np.random.default_rng(123).choice(n, 3000, replace=False)
    idx = np.concatenate([idx, [0, n - 1]])
    ref = om.state_rhoe(st["rho"][idx], st["e"][idx], np.ascontiguousarray(Y[:, idx]))
    gs = {k: v[idx] for k, v in g.items()}
    worst = compare(gs, ref, 1, FP64_RTOL)
    _report("rhoey fp64 128^3 sampled", worst)
    assert max(worst.values()) <= 1.0, worst
    # properties that hold at every cell of the field
    assert np.all(g["status"] == 0)
    assert np.max(np.abs(g["T"] / T - 1)) < 1e-10
    assert np.all(np.isfinite(g["mu"])) and np.all(g["mu"] > 0) and np.all(g["lambda"] > 0)
    del g
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ mixed precision

def test_mixed_precision_error_report(props, orc, sp8, kij8):
    P, T, Y = synth.flame_field(24, seed=1)
    n = T.size
    om = orc.Mech(sp8, kij8)
    st = om.state_PT(P, T, Y, transport=False)
    ref = om.state_rhoe(st["rho"], st["e"], Y)
    gm = props.Mechanism(sp8, kij8)
    g = run_gpu(props, gm, props.RHOEY, props.MIXED, n,
                {"rho": st["rho"], "e": st["e"], "Y": Y, "T_guess": synth.temperature_guess(T)},
                fields=FIELDS + ("iters",))
    stats = rel_err_stats(g, ref)
    assert np.all(g["status"] == 0), np.unique(g["status"])
    assert g["iters"].max() <= 8, np.bincount(g["iters"].astype(np.int64))
    print("\n[mixed rhoey] max/rms rel err: " + ", ".join(f"{k}={v[0]:.2e}/{v[1]:.2e}" for k, v in stats.items()))
    for f in ("rho", "h", "cp", "T", "P", "Z", "e", "c", "mu", "lambda"):
        assert stats[f][0] <= MIXED_RTOL, (f, stats[f])
    gp = run_gpu(props, gm, props.PTY, props.MIXED, n, {"P": P, "T": T, "Y": Y})
    refp = om.state_PT(P, T, Y)
    statsp = rel_err_stats(gp, refp)
    print("[mixed pty] max/rms rel err: " + ", ".join(f"{k}={v[0]:.2e}/{v[1]:.2e}" for k, v in statsp.items()))
    for f in ("rho", "h", "cp", "c", "mu", "lambda"):
        assert statsp[f][0] <= MIXED_RTOL, (f, statsp[f])


@pytest.mark.parametrize("mode", ["PTY", "RHOEY", "HPY"])
def test_mixed_precision_ragged_launch(props, orc, sp8, kij8, mode):
    """Mixed precision (launched in blocks of 64 lanes) on cell counts that end inside a
    block, and on one cell: every cell is written, each within the mixed-precision bar of the
    FP64 oracle (outputs are pre-filled with a sentinel, status with 255)."""
    P, T, Y = synth.flame_field(16, seed=12)
    om = orc.Mech(sp8, kij8)
    gm = props.Mechanism(sp8, kij8)
    for n in (T.size - 37, 65, 1):
        Pn, Tn, Yn = P[:n], T[:n], np.ascontiguousarray(Y[:, :n])
        st = om.state_PT(Pn, Tn, Yn, transport=(mode == "PTY"))
        if mode == "PTY":
            ref, inputs = st, {"P": Pn, "T": Tn, "Y": Yn}
        elif mode == "RHOEY":
            ref = om.state_rhoe(st["rho"], st["e"], Yn)
            inputs = {"rho": st["rho"], "e": st["e"], "Y": Yn, "T_guess": synth.temperature_guess(Tn)}
        else:
            ref = om.state_hP(st["h"], Pn, Yn)
            inputs = {"h": st["h"], "P": Pn, "Y": Yn, "T_guess": synth.temperature_guess(Tn)}
        g = run_gpu(props, gm, getattr(props, mode), props.MIXED, n, inputs)
        assert np.all(g["status"] == 0), (n, np.unique(g["status"]))
        stats = rel_err_stats(g, ref)
        for f, (mx, _) in stats.items():
            assert mx <= MIXED_RTOL, (mode, n, f, mx)


# ------------------------------------------------------------------ edge cases

def test_three_root_gibbs_selection(props, orc):
    """Subcritical O2 and CH4 around their PR saturation pressure: three physical roots,
    vapour root below P_sat, liquid root above (both sides agree cell by cell)."""
    for name, T0, ps in (("O2", 120.0, 1.02678e6), ("CH4", 150.0, 1.04691e6)):
        sp = synth.load_species([name])
        P = ps * np.array([0.5, 0.9, 0.99, 0.999, 1.001, 1.01, 1.1, 1.5])
        T = np.full(P.size, T0)
        Y = np.ones((1, P.size))
        ref = orc.Mech(sp).state_PT(P, T, Y)
        g = run_gpu(props, props.Mechanism(sp), props.PTY, props.FP64, P.size, {"P": P, "T": T, "Y": Y})
        assert np.array_equal(g["status"], ref["status"]), (g["status"], ref["status"])
        assert np.any(ref["status"] & 8)
        worst = compare(g, ref, 0, FP64_RTOL)
        assert max(worst.values()) <= 1.0, worst


def test_gibbs_tie_at_the_saturation_pressure(props, orc):
    """Pure O2 at 120 K: at the pressure where the two residual Gibbs energies cross (found
    by bisection on their difference with the oracle) both sides flag a tie and take the
    vapour-like root; five parts in 1e12 to either side neither flags one, and the roots
    differ (vapour below, liquid above)."""
    sp = synth.load_species(["O2"])
    om = orc.Mech(sp)
    T = 120.0
    am, _, _, bm = om.mix(np.array([1.0]), T)
    R = 8.31446261815324

    def dg(P):
        A, B = am * P / (R * T) ** 2, bm * P / (R * T)
        r = orc.cubic_roots(A, B)
        return orc.gdep_RT(r[0], A, B) - orc.gdep_RT(r[-1], A, B)

    lo, hi = 1.0e6, 1.05e6
    assert dg(lo) > 0 > dg(hi)
    while np.nextafter(lo, np.inf) < hi:
        mid = 0.5 * (lo + hi)
        if mid in (lo, hi):
            break
        lo, hi = (mid, hi) if dg(mid) > 0 else (lo, mid)
    P = np.array([lo, lo * (1 - 5e-12), lo * (1 + 5e-12)])
    Tv = np.full(3, T)
    Y = np.ones((1, 3))
    ref = om.state_PT(P, Tv, Y)
    g = run_gpu(props, props.Mechanism(sp), props.PTY, props.FP64, 3, {"P": P, "T": Tv, "Y": Y})
    assert np.array_equal(g["status"], ref["status"]), (g["status"], ref["status"])
    assert ref["status"][0] & 16 and not (ref["status"][1] & 16) and not (ref["status"][2] & 16)
    assert g["Z"][0] > 0.3 and g["Z"][1] > 0.3 and g["Z"][2] < 0.3
    worst = compare(g, ref, 0, FP64_RTOL)
    assert max(worst.values()) <= 1.0, worst


def test_nonphysical_and_bracket_flags(props, orc, sp8, kij8):
    n = 8
    Y = np.zeros((8, n))
    Y[1] = 1.0
    rho = np.array([100.0, 100.0, -1.0, 100.0, 100.0, 100.0, 1e6, 100.0])
    e = np.array([5e7, -5e7, 0.0, 0.0, np.nan, 0.0, 0.0, -1e5])
    Y[:, 5] = 0.0
    Y[1, 5] = 0.9          # sum Y != 1
    Y[:, 7] = 0.0
    Y[0, 7], Y[1, 7] = -0.5, 1.5   # negative mass fraction
    ref = orc.Mech(sp8, kij8).state_rhoe(rho, e, Y)
    g = run_gpu(props, props.Mechanism(sp8, kij8), props.RHOEY, props.FP64, n, {"rho": rho, "e": e, "Y": Y})
    assert np.array_equal(g["status"], ref["status"]), (g["status"], ref["status"])
    for f in FIELDS:
        assert np.array_equal(np.isnan(g[f]), np.isnan(ref[f])), f
    P = np.array([1e7, -1.0, 1e7, np.nan])
    T = np.array([300.0, 300.0, 0.0, 300.0])
    Yp = np.zeros((8, 4))
    Yp[0] = 1.0
    refp = orc.Mech(sp8, kij8).state_PT(P, T, Yp)
    gp = run_gpu(props, props.Mechanism(sp8, kij8), props.PTY, props.FP64, 4, {"P": P, "T": T, "Y": Yp})
    assert np.array_equal(gp["status"], refp["status"])


def test_newton_iteration_limit_flag(props, orc, sp8, kij8):
    P, T, Y = synth.flame_field(6, seed=3)
    st = orc.Mech(sp8, kij8).state_PT(P, T, Y, transport=False)
    m = props.Mechanism(sp8, kij8)
    m.set_newton(max_iter=1)
    g = run_gpu(props, m, props.RHOEY, props.FP64, T.size, {"rho": st["rho"], "e": st["e"], "Y": Y})
    assert np.all(g["status"] & 2)
    m.set_newton(100, 1e-10)
    g = run_gpu(props, m, props.RHOEY, props.FP64, T.size, {"rho": st["rho"], "e": st["e"], "Y": Y})
    assert np.all(g["status"] == 0)


@pytest.mark.parametrize("ns", [1, 3, 5, 8])
def test_species_counts_and_padding(props, orc, sp8, ns):
    sp = sp8[:ns]
    rng = np.random.default_rng(ns)
    n = 1000
    Y = rng.dirichlet(np.ones(ns), n).T.copy()
    P = rng.uniform(1e6, 2e7, n)
    T = rng.uniform(200.0, 2500.0, n)
    kij = synth.synthetic_kij(ns, seed=ns)
    ref = orc.Mech(sp, kij).state_PT(P, T, Y)
    g = run_gpu(props, props.Mechanism(sp, kij), props.PTY, props.FP64, n, {"P": P, "T": T, "Y": Y})
    # uniform compositions with H2 (ns > 5) reach Chung's singular acentric factor: the
    # transport outputs carry the correlation's own condition number
    kmu, klam = chung_kappa(sp, Y)
    worst = compare(g, ref, 0, FP64_RTOL, extra={"mu": kmu, "lambda": klam})
    _report(f"species {ns}, max kappa_mu {kmu.max():.3g}", worst)
    assert max(worst.values()) <= 1.0, worst


def test_null_outputs_and_empty_launch(props, orc, sp8, kij8):
    import torch
    P, T, Y = synth.flame_field(5, seed=2)
    n = T.size
    ref = orc.Mech(sp8, kij8).state_PT(P, T, Y)
    m = props.Mechanism(sp8, kij8)
    g = run_gpu(props, m, props.PTY, props.FP64, n, {"P": P, "T": T, "Y": Y},
                fields=("rho", "h"), want_status=False)
    worst = compare(g, ref, 0, FP64_RTOL, fields=("rho", "h"))
    assert max(worst.values()) <= 1.0
    props.pr(m, props.PTY, props.FP64, {"P": None, "T": None, "Y": torch.zeros(1, device="cuda:0", dtype=torch.float64)}, {}, 0)


def test_invalid_arguments_raise(props, sp8):
    with pytest.raises(props.PropsError):
        props.Mechanism(sp8 + sp8[:1])           # 9 species > PROPS_MAX_SPECIES
    bad = [dict(s) for s in sp8[:2]]
    bad[1]["Tmid"] = 1200.0
    with pytest.raises(props.PropsError):
        props.Mechanism(bad)
    with pytest.raises(props.PropsError):
        props.Mechanism(sp8[:2], [[0.0, 0.1], [0.2, 0.0]])   # asymmetric k_ij
    m = props.Mechanism(sp8[:2])
    with pytest.raises(props.PropsError):
        props.pr(m, props.PTY, props.FP64, {}, {}, 10)        # missing inputs
    with pytest.raises(props.PropsError):
        props.pr(m, 7, props.FP64, {}, {}, 10)


def test_deterministic_bitwise(props, sp8, kij8, orc):
    P, T, Y = synth.flame_field(16, seed=5)
    st = orc.Mech(sp8, kij8).state_PT(P, T, Y, transport=False)
    m = props.Mechanism(sp8, kij8)
    inp = {"rho": st["rho"], "e": st["e"], "Y": Y, "T_guess": synth.temperature_guess(T)}
    a = run_gpu(props, m, props.RHOEY, props.FP64, T.size, inp)
    b = run_gpu(props, m, props.RHOEY, props.FP64, T.size, inp)
    for f in FIELDS:
        assert np.array_equal(a[f].view(np.int64), b[f].view(np.int64)), f


def test_chung_near_singular_mixture(props, orc, sp8):
    """H2/CH4 mixtures sweep the pseudo-mixture acentric factor through the value where
    Chung's density-function denominator E1 E4 + E2 + E3 vanishes; both sides then agree to
    1e-12 scaled by the denominator's condition number (chung_kappa)."""
    sp = [sp8[0], sp8[5]]
    n = 2000
    xh2 = np.linspace(0.02, 0.98, n)
    W = np.array([s["W"] for s in sp])
    Y = np.stack([(1 - xh2) * W[0], xh2 * W[1]])
    Y /= Y.sum(0, keepdims=True)
    P = np.full(n, 5e6)
    T = np.full(n, 900.0)
    ref = orc.Mech(sp).state_PT(P, T, Y)
    g = run_gpu(props, props.Mechanism(sp), props.PTY, props.FP64, n, {"P": P, "T": T, "Y": Y})
    kmu, klam = chung_kappa(sp, Y)
    for f, kappa in (("mu", kmu), ("lambda", klam)):
        err = np.abs(g[f] - ref[f]) / np.abs(ref[f])
        ok = np.isfinite(ref[f])
        print(f"\n[chung near-singular] {f}: max kappa {kappa.max():.3g}, worst err/tol "
              f"{float(np.max(err[ok] / (FP64_RTOL * kappa[ok]))):.3g}", flush=True)
        assert np.all(err[ok] <= FP64_RTOL * kappa[ok]), (f, float(np.max(err[ok] / (FP64_RTOL * kappa[ok]))))
