"""Surrogate input features of the pressure-based solver — TEST INFRASTRUCTURE ONLY.

Plain numpy definitions, independent of the GPU library:
  - Bilger's mixture fraction (the paper's third surrogate input, Section 4.1) from element
    mass fractions Y_e = sum_i Y_i n_{e,i} A_e / W_i with the coupling function
    beta = 2 Y_C / A_C + Y_H / (2 A_H) - Y_O / A_O, normalised between the pure fuel and
    the pure oxidizer streams: Z = (beta - beta_ox) / (beta_fuel - beta_ox);
  - the Box-Cox transform (Section 4.2) BC(Z) = (Z^lambda - 1) / lambda (lambda > 0), with
    Z clamped below at 0 first.
"""
import numpy as np

# standard atomic masses, kg/mol (IUPAC conventional values)
ATOMIC_MASS = {"C": 12.011e-3, "H": 1.008e-3, "O": 15.999e-3}


def element_mass_fractions(species, Y):
    """Y: [ns, n] mass fractions -> dict element -> [n] element mass fraction."""
    Y = np.asarray(Y, dtype=np.float64)
    out = {}
    for e, A in ATOMIC_MASS.items():
        w = np.array([s["atoms"][e] * A / s["W"] for s in species])
        out[e] = (w[:, None] * Y).sum(0)
    return out


def coupling_beta(species, Y):
    Ye = element_mass_fractions(species, Y)
    return 2.0 * Ye["C"] / ATOMIC_MASS["C"] + Ye["H"] / (2.0 * ATOMIC_MASS["H"]) - Ye["O"] / ATOMIC_MASS["O"]


def bilger_Z(species, Y, fuel, oxidizer):
    """Bilger mixture fraction between the pure species `fuel` and `oxidizer` (indices)."""
    ns = len(species)
    unit = np.eye(ns)
    b = coupling_beta(species, Y)
    bf = coupling_beta(species, unit[:, [fuel]])[0]
    bo = coupling_beta(species, unit[:, [oxidizer]])[0]
    return (b - bo) / (bf - bo)


def box_cox(Z, lam):
    if not (0.0 < lam <= 1.0):
        raise ValueError("0 < lambda <= 1")
    Zc = np.maximum(np.asarray(Z, dtype=np.float64), 0.0)
    return (Zc ** lam - 1.0) / lam


def hpz_features(species, fuel, oxidizer, lam, h, P, Y, nin=10):
    """[nin, n] features: h, P, BC(Z), then zeros."""
    h = np.asarray(h, dtype=np.float64)
    X = np.zeros((nin, h.size))
    X[0] = h
    X[1] = P
    X[2] = box_cox(bilger_Z(species, Y, fuel, oxidizer), lam)
    return X
