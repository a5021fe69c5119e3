"""Write ``species_ch4o2_8.json``: the species constants for the CH4/O2 flame mixture.

The paper takes all species data from Cantera (Section 2) and prints none of it: no
critical constants, no acentric factors, no NASA-7 coefficients. No thermochemical
database is available to this project, so this script *derives* the ideal-gas part from
first principles and records where every other number comes from:

* Critical constants, acentric factor, critical volume, dipole moment and the Chung
  association factor are textbook values (Poling, Prausnitz & O'Connell, *The Properties
  of Gases and Liquids*, 5th ed., Appendix A and Table 9-1), typed in below.
* The NASA-7 polynomials are least-squares fits (two ranges, T_mid = 1000 K, c_p and its
  slope continuous at T_mid) to the rigid-rotor / harmonic-oscillator ideal-gas heat
  capacity: translation 5/2 R, rotation R (linear) or 3/2 R (nonlinear), one Einstein
  term per vibrational mode, plus the low-lying electronic levels of O2 and OH.
  a6 is set so that h(298.15 K) equals the standard enthalpy of formation and h is
  continuous at T_mid.  a7 (entropy) is not used by the property path and is left 0.
  Expect 1-3 % deviation from JANAF tables at high T (no anharmonicity).

* Dipole moments are written as 0 ("dipole"), with the physical value kept under
  "dipole_physical".  Chung's pseudo-mixture correlation is singular for polar mixtures:
  with H2O at 1.8 D, a mixture holding ~10-30 % H2O reaches a reduced pseudo-dipole
  mu_rm^4 ~ 0.15-0.2 at which the denominator E1 E4 + E2 + E3 of its density function G2
  passes through zero and the viscosity changes sign.  The non-polar treatment keeps the
  association factor of H2O and is regular everywhere in the flame.

The resulting file is an *input* to both the GPU library and the CPU oracle, exactly like
a mechanism file handed to Cantera; each side derives its own constants from it.

Run: ``python synth/make_species.py`` (rewrites the JSON next to this file).
"""
import json
import os

import numpy as np

R = 8.31446261815324          # J/(mol K)
HC_K = 1.438776877            # second radiation constant h c / k_B in cm K
T_REF = 298.15
T_MID = 1000.0
T_LO = (100.0, T_MID)         # the flame field reaches 120 K: fit below the usual 200 K
T_HI = (T_MID, 6000.0)

# name, W [kg/mol], Tc [K], Pc [Pa], Vc [m^3/mol], omega, dipole [debye], kappa (Chung),
# dHf(298.15) [J/mol], linear?, vibrational wavenumbers [cm^-1] (repeated per degeneracy),
# electronic levels [(cm^-1, degeneracy)]
SPECIES = [
    ("CH4", 16.043e-3, 190.56, 4.599e6, 98.6e-6, 0.0115, 0.0, 0.0, -74.87e3, False,
     [2917.0, 1534.0, 1534.0, 3019.0, 3019.0, 3019.0, 1306.0, 1306.0, 1306.0], [(0.0, 1)]),
    ("O2", 31.998e-3, 154.58, 5.043e6, 73.4e-6, 0.0222, 0.0, 0.0, 0.0, True,
     [1580.0], [(0.0, 3), (7918.1, 2), (13195.1, 1)]),
    ("CO2", 44.010e-3, 304.12, 7.374e6, 94.07e-6, 0.225, 0.0, 0.0, -393.51e3, True,
     [1333.0, 667.0, 667.0, 2349.0], [(0.0, 1)]),
    ("H2O", 18.015e-3, 647.14, 22.064e6, 55.95e-6, 0.344, 1.8, 0.076, -241.83e3, False,
     [3657.0, 1595.0, 3756.0], [(0.0, 1)]),
    ("CO", 28.010e-3, 132.85, 3.494e6, 93.1e-6, 0.045, 0.1, 0.0, -110.53e3, True,
     [2170.0], [(0.0, 1)]),
    ("H2", 2.016e-3, 33.19, 1.313e6, 64.2e-6, -0.216, 0.0, 0.0, 0.0, True,
     [4401.0], [(0.0, 1)]),
    # OH is a radical with no measurable critical point: it borrows the critical
    # constants of H2O, with its own molar mass, zero dipole and zero association.
    ("OH", 17.007e-3, 647.14, 22.064e6, 55.95e-6, 0.344, 0.0, 0.0, 37.36e3, True,
     [3738.0], [(0.0, 2), (139.7, 2)]),
    ("N2", 28.014e-3, 126.20, 3.398e6, 90.1e-6, 0.037, 0.0, 0.0, 0.0, True,
     [2359.0], [(0.0, 1)]),
]


def cp_rrho_over_R(T, linear, vib, elec):
    """Ideal-gas c_p/R from translation + rotation + harmonic vibration + electronic levels."""
    T = np.asarray(T, dtype=np.float64)
    cp = 2.5 + (1.0 if linear else 1.5) + np.zeros_like(T)
    for nu in vib:
        x = HC_K * nu / T
        ex = np.exp(-x)
        cp = cp + x * x * ex / (1.0 - ex) ** 2
    if len(elec) > 1:
        eps = np.array([e for e, _ in elec])[:, None] * HC_K / T[None, :]
        g = np.array([d for _, d in elec], dtype=np.float64)[:, None]
        w = g * np.exp(-eps)
        q = w.sum(0)
        m1 = (w * eps).sum(0) / q
        m2 = (w * eps * eps).sum(0) / q
        cp = cp + (m2 - m1 * m1)
    return cp


def fit_nasa7(linear, vib, elec, dhf):
    """Joint constrained least-squares fit of the two c_p ranges, then a6 from h."""
    tl = np.linspace(*T_LO, 400)
    th = np.linspace(*T_HI, 600)
    basis = lambda T: np.stack([T ** k for k in range(5)], axis=1)   # noqa: E731
    Al, Ah = basis(tl), basis(th)
    yl, yh = cp_rrho_over_R(tl, linear, vib, elec), cp_rrho_over_R(th, linear, vib, elec)
    # unknowns x = [lo(5), hi(5)]; constraints: cp and dcp/dT equal at T_mid
    A = np.zeros((len(tl) + len(th), 10))
    A[:len(tl), :5] = Al
    A[len(tl):, 5:] = Ah
    y = np.concatenate([yl, yh])
    bm = basis(np.array([T_MID]))[0]
    dbm = np.array([0.0, 1.0, 2 * T_MID, 3 * T_MID ** 2, 4 * T_MID ** 3])
    C = np.zeros((2, 10))
    C[0, :5], C[0, 5:] = bm, -bm
    C[1, :5], C[1, 5:] = dbm, -dbm
    # scale columns for conditioning
    s = np.concatenate([1.0 / np.array([1, 1e3, 1e6, 1e9, 1e12])] * 2)
    As, Cs = A * s, C * s
    K = np.block([[As.T @ As, Cs.T], [Cs, np.zeros((2, 2))]])
    rhs = np.concatenate([As.T @ y, np.zeros(2)])
    x = np.linalg.solve(K, rhs)[:10] * s
    lo, hi = x[:5], x[5:]

    def h_RT_poly(a, T):
        return a[0] + a[1] * T / 2 + a[2] * T ** 2 / 3 + a[3] * T ** 3 / 4 + a[4] * T ** 4 / 5

    a6_lo = dhf / R - T_REF * h_RT_poly(lo, T_REF)
    h_mid = T_MID * h_RT_poly(lo, T_MID) + a6_lo
    a6_hi = h_mid - T_MID * h_RT_poly(hi, T_MID)
    lo7 = list(lo) + [a6_lo, 0.0]
    hi7 = list(hi) + [a6_hi, 0.0]
    err = max(np.max(np.abs(Al @ lo - yl) / yl), np.max(np.abs(Ah @ hi - yh) / yh))
    return lo7, hi7, err


# atoms per molecule (C, H, O, N): the element balance behind Bilger's mixture fraction
ATOMS = {"CH4": (1, 4, 0, 0), "O2": (0, 0, 2, 0), "CO2": (1, 0, 2, 0), "H2O": (0, 2, 1, 0),
         "CO": (1, 0, 1, 0), "H2": (0, 2, 0, 0), "OH": (0, 1, 1, 0), "N2": (0, 0, 0, 2)}


def main():
    out = {
        "description": "CH4/O2 supercritical flame mixture, 8 species; SI units. "
                       "Critical data: Poling, Prausnitz & O'Connell 5th ed. App. A / Table 9-1. "
                       "NASA-7: rigid-rotor harmonic-oscillator fits written by synth/make_species.py.",
        "R": R,
        "species": [],
    }
    for (name, W, Tc, Pc, Vc, om, dip, kap, dhf, linear, vib, elec) in SPECIES:
        lo, hi, err = fit_nasa7(linear, vib, elec, dhf)
        out["species"].append({
            "name": name, "W": W, "Tc": Tc, "Pc": Pc, "Vc": Vc, "omega": om,
            "dipole": 0.0, "dipole_physical": dip, "kappa": kap, "dhf298": dhf, "Tmid": T_MID,
            "nasa_lo": lo, "nasa_hi": hi, "fit_max_rel_err": err,
            "atoms": dict(zip(("C", "H", "O", "N"), ATOMS[name])),
            "rrho": {"linear": linear, "vib_cm": vib, "elec": elec},
        })
        print(f"{name:4s} fit max rel err {err:.2e}  cp(298)/R={cp_rrho_over_R(np.array([T_REF]), linear, vib, elec)[0]:.4f}")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "species_ch4o2_8.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
