"""Seeded synthetic inputs shared by the GPU path's callers and by the CPU oracle's tests.

This module holds the *inputs* only: species constants (a JSON mechanism file), state
fields shaped like the paper's supercritical CH4/LOX Taylor-Green flame (Section 3), the
binary-interaction matrix, training-sample states and serving request traces.  It holds
none of the property method's arithmetic (no equation of state, no thermochemistry, no
transport): fields are built from temperature, pressure and mass fractions only, and the
densities/energies a solver would carry are produced by whichever property engine the
caller is testing or timing.

All draws use numpy's PCG64 (``np.random.default_rng(seed)``) in the order documented on
each function, so a seed fixes the field bit for bit.
"""
import json
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SPECIES_FILE = os.path.join(_HERE, "species_ch4o2_8.json")
FLAME_SPECIES = ("CH4", "O2", "CO2", "H2O", "CO", "H2", "OH", "N2")

# Taylor-Green flame geometry (Section 3): L = 2 pi L0, L0 = 0.03 mm, u0 = 4 m/s.
L0 = 3.0e-5
L_BOX = 2.0 * math.pi * L0
P_REF = 10.0e6


def load_species(names=None, path=SPECIES_FILE):
    """Return a list of plain dicts (SI units) for the requested species, in that order."""
    with open(path) as f:
        data = json.load(f)
    table = {s["name"]: s for s in data["species"]}
    names = list(names) if names is not None else [s["name"] for s in data["species"]]
    return [dict(table[n]) for n in names]


def synthetic_kij(ns, seed=7, kmax=0.1):
    """Dense symmetric binary-interaction matrix, k_ij ~ U[0, kmax], zero diagonal.

    The paper prints no k_ij; a dense non-zero matrix exercises the full N_s x N_s
    mixing sums instead of the rank-1 k = 0 shortcut.
    """
    rng = np.random.default_rng(seed)
    k = rng.uniform(0.0, kmax, size=(ns, ns))
    k = np.triu(k, 1)
    return k + k.T


def cells_uniform(n=4096, seed=0):
    """Independent two-species cells (CH4, O2): draws P, then T, then Y_CH4.

    P ~ U[5, 15] MPa, T ~ U[100, 1000] K, Y_CH4 ~ U[0, 1], Y_O2 = 1 - Y_CH4.
    Returns (P[n], T[n], Y[2, n]) float64, Y species-major.
    """
    rng = np.random.default_rng(seed)
    P = rng.uniform(5.0e6, 15.0e6, n)
    T = rng.uniform(100.0, 1000.0, n)
    y = rng.uniform(0.0, 1.0, n)
    return P, T, np.stack([y, 1.0 - y])


def _stoich(species):
    W = {s["name"]: s["W"] for s in species}
    wf = W["CH4"] + 2.0 * W["O2"]
    return W["CH4"] / wf, W["CO2"] / wf, 2.0 * W["H2O"] / wf


def flame_state(xi, species):
    """Burke-Schumann-like composition and temperature for CH4 + 2 O2 -> CO2 + 2 H2O.

    Pure fuel at xi = 1 (300 K), pure oxygen at xi = 0 (120 K), complete products at the
    stoichiometric mixture fraction (3000 K); T piecewise linear in xi between them.
    Minor species CO, H2, OH follow a Gaussian bump around xi_st taken from CO2/H2O in
    proportion; N2 is a 1e-3 trace.  Returns (T, Y[8, ...]) before noise and
    renormalisation.
    """
    xi = np.asarray(xi, dtype=np.float64)
    xst, yco2, yh2o = _stoich(species)
    lean = xi <= xst
    prod = np.where(lean, xi / xst, (1.0 - xi) / (1.0 - xst))
    Y = np.zeros((8,) + xi.shape)
    Y[0] = np.where(lean, 0.0, (xi - xst) / (1.0 - xst))
    Y[1] = np.where(lean, 1.0 - xi / xst, 0.0)
    Y[2] = yco2 * prod
    Y[3] = yh2o * prod
    bump = np.exp(-((xi - xst) / 0.05) ** 2)
    minor = np.stack([0.04 * bump, 0.002 * bump, 0.01 * bump])
    take = minor.sum(0)
    pr = Y[2] + Y[3]
    frac = np.divide(take, pr, out=np.zeros_like(pr), where=pr > 0)
    frac = np.minimum(frac, 1.0)
    Y[2] *= 1.0 - frac
    Y[3] *= 1.0 - frac
    Y[4], Y[5], Y[6] = minor * np.where(pr > 0, 1.0, 0.0)
    Y[7] = 1.0e-3
    T = np.where(lean, 120.0 + (3000.0 - 120.0) * xi / xst,
                 3000.0 + (300.0 - 3000.0) * (xi - xst) / (1.0 - xst))
    return T, Y


def _xi_from_points(x, y, z):
    # one reference time of Taylor-Green advection at u0 (the 3D form of Eqs. 2-3)
    xp = x + L0 * np.sin(x / L0) * np.cos(y / L0) * np.cos(z / L0)
    d = 0.05 * L_BOX
    return 0.5 * (np.tanh((xp - L_BOX / 4) / d) - np.tanh((xp - 3 * L_BOX / 4) / d))


def _noise(rng, T, Y, npts):
    """Draw order: species noise (8 x n normal, clipped at +-3), then pressure U(-1, 1)."""
    g = np.clip(rng.standard_normal((8, npts)), -3.0, 3.0)
    Y = Y * (1.0 + 0.01 * g)
    Y = np.maximum(Y, 0.0)
    Y = Y / Y.sum(0, keepdims=True)
    u = rng.uniform(-1.0, 1.0, npts)
    P = P_REF * (1.0 + 0.01 * u)
    return P, T, Y


def flame_field(res=128, seed=1, species=None):
    """The Taylor-Green flame field on a res^3 grid of cell centres over [0, L)^3.

    Cells are ordered x fastest.  Returns (P[n], T[n], Y[8, n]) float64, n = res^3.
    """
    species = species or load_species(FLAME_SPECIES)
    c = (np.arange(res) + 0.5) * (L_BOX / res)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    xi = _xi_from_points(x.ravel(), y.ravel(), z.ravel())
    T, Y = flame_state(xi, species)
    rng = np.random.default_rng(seed)
    return _noise(rng, T, Y, xi.size)


def flame_field_rows(res, row0, nrows, seed=1, species=None):
    """Rows [row0, row0 + nrows) of ``flame_field(res, seed)`` without building the rest.

    A 'row' is one x-line of ``res`` cells.  The noise of a row depends only on the seed
    and the row index, so the pieces differ from ``flame_field``; use this for fields too
    large to hold at once (it is seeded per row: ``seed * 1_000_003 + row``).
    """
    species = species or load_species(FLAME_SPECIES)
    c = (np.arange(res) + 0.5) * (L_BOX / res)
    Ps, Ts, Ys = [], [], []
    for r in range(row0, row0 + nrows):
        iz, iy = divmod(r, res)
        x = c
        yv = np.full(res, c[iy])
        zv = np.full(res, c[iz])
        xi = _xi_from_points(x, yv, zv)
        T, Y = flame_state(xi, species)
        rng = np.random.default_rng(seed * 1_000_003 + r)
        P, T, Y = _noise(rng, T, Y, res)
        Ps.append(P), Ts.append(T), Ys.append(Y)
    return np.concatenate(Ps), np.concatenate(Ts), np.concatenate(Ys, axis=1)


def temperature_guess(T_true, seed=11, rel=0.01):
    """A previous-iterate style guess T_true * (1 + rel * g), g ~ N(0, 1) clipped at +-3."""
    rng = np.random.default_rng(seed)
    g = np.clip(rng.standard_normal(T_true.shape), -3.0, 3.0)
    return T_true * (1.0 + rel * g)


def training_states(n, seed=3, species=None, jitter_a2=50.0):
    """(P, T, Y) training states drawn like the flame field, with the paper's Eq. 4 jitter.

    Draw order: positions (3 x n uniform in the box), species/pressure noise as in the
    field, then the jitter a1 ~ U(-1, 1) for T, then for P, then a multiplicative
    Y jitter (8 x n, U(-1, 1) / a2).  Each variable t = c + a1 (max c - min c) / a2.
    Samples violating the physical constraints (Y in [0, 1], T in [100, 3100] K, P > 0)
    are redrawn.  Returns float64 arrays (P[n], T[n], Y[8, n]).
    """
    species = species or load_species(FLAME_SPECIES)
    rng = np.random.default_rng(seed)
    out_P, out_T, out_Y = [], [], []
    have = 0
    while have < n:
        m = int((n - have) * 1.05) + 16
        pts = rng.uniform(0.0, L_BOX, size=(3, m))
        xi = _xi_from_points(pts[0], pts[1], pts[2])
        T, Y = flame_state(xi, species)
        P, T, Y = _noise(rng, T, Y, m)
        a1T = rng.uniform(-1.0, 1.0, m)
        a1P = rng.uniform(-1.0, 1.0, m)
        aY = rng.uniform(-1.0, 1.0, (8, m))
        T = T + a1T * (3000.0 - 120.0) / jitter_a2
        P = P + a1P * (0.02 * P_REF) / jitter_a2
        Y = Y * (1.0 + aY / jitter_a2)
        Y = np.maximum(Y, 0.0)
        Y = Y / Y.sum(0, keepdims=True)
        ok = (T >= 100.0) & (T <= 3100.0) & (P > 0) & np.all((Y >= 0) & (Y <= 1), axis=0)
        out_P.append(P[ok]), out_T.append(T[ok]), out_Y.append(Y[:, ok])
        have += int(ok.sum())
    P = np.concatenate(out_P)[:n]
    T = np.concatenate(out_T)[:n]
    Y = np.concatenate(out_Y, axis=1)[:, :n]
    return P, T, Y


def serving_trace(n_sub=64, reqs_per_sub=50, seed=5, nmin=4096, nmax=2_097_152, rate=None):
    """Request trace for concurrent subdomains.

    Draw order: subdomain sizes n_k = round(exp(U[ln nmin, ln nmax])), then for each
    subdomain in turn its exponential inter-arrival gaps (mean n_sub / rate seconds).
    Returns a list of (t_arrival_s, subdomain, n_cells) sorted by arrival time.
    """
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_sub))).astype(np.int64)
    rate = rate if rate is not None else 100.0
    reqs = []
    for k in range(n_sub):
        gaps = rng.exponential(n_sub / rate, reqs_per_sub)
        t = np.cumsum(gaps)
        reqs.extend((float(ti), k, int(sizes[k])) for ti in t)
    reqs.sort()
    return reqs, sizes
