"""Helpers for GPU-vs-oracle parity tests: run the HIP path through the C ABI and
compare element by element with condition-scaled tolerances."""
import numpy as np

R = 8.31446261815324
FIELDS = ("T", "P", "Z", "rho", "h", "e", "cp", "c", "mu", "lambda")


def run_gpu(props, mech, mode, prec, n, inputs, fields=FIELDS, stream=None, want_status=True, ns=None):
    """Copy numpy inputs to the device, call props_pr, return numpy outputs + status
    (hRT, [ns][n], needs ns)."""
    import torch
    dev = torch.device("cuda:0")
    tin = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(dev)
           for k, v in inputs.items() if v is not None}

    def alloc(k):
        if k == "iters":
            return torch.zeros(n, dtype=torch.uint8, device=dev)
        shape = (ns, n) if k == "hRT" else (n,)
        return torch.full(shape, -12345.0, dtype=torch.float64, device=dev)

    tout = {k: alloc(k) for k in fields}
    st = torch.full((n,), 255, dtype=torch.uint8, device=dev) if want_status else None
    props.pr(mech, mode, prec, tin, tout, n, status=st, stream=stream)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in tout.items()}
    if want_status:
        out["status"] = st.cpu().numpy().astype(np.int32)
    return out


def cell_kappa(ref, mode):
    """Per-cell condition number bounding the relative rounding error of the outputs.

    kappa_cp: cancellation in (dP/dv)_T and in the c_p correction; kappa_Z (P,T mode):
    polynomial root condition; kappa_T (rho,e mode): relative sensitivity of T to e; and
    the cancellation in Eq. (1) itself, (RT/(v-b) + a/(v^2+2bv-b^2)) / |P|.
    """
    v, T, am, bm = ref["v"], ref["T"], ref["am"], ref["bm"]
    den = v * v + 2 * bm * v - bm * bm
    kP = (R * T / (v - bm) + am / den) / np.abs(ref["P"])
    k = np.maximum.reduce([np.ones_like(T), ref["kappa_cp"], kP])
    if mode == 0:
        k = np.maximum(k, ref["kappa_Z"])
    else:
        k = np.maximum(k, ref["kappa_T"] * kP)
    return k


def compare(gpu, ref, mode, rtol, fields=FIELDS, mask=None, kappa=True, extra=None, scales=None):
    """Return {field: worst err/tol}; h and e are compared against their sums of
    magnitudes (they cross zero), everything else relative to itself unless `scales` gives
    a per-cell magnitude for it.  extra: optional {field: per-cell factor} multiplying that
    field's condition number."""
    k0 = cell_kappa(ref, mode) if kappa else np.ones(len(ref))
    worst = {}
    for f in fields:
        k = k0 * extra[f] if extra and f in extra else k0
        g = gpu[f]
        r = ref["lambda"] if f == "lambda" else ref[f]
        if scales and f in scales:
            scale = scales[f]
        elif f == "h":
            scale = ref["h_scale"]
        elif f == "e":
            scale = ref["e_scale"]
        else:
            scale = np.abs(r)
        tol = rtol * k * scale
        both_nan = np.isnan(g) & np.isnan(r)
        err = np.where(both_nan, 0.0, np.abs(g - r))
        err = np.where(np.isnan(err), np.inf, err)
        ratio = err / np.maximum(tol, 1e-300)
        if mask is not None:
            ratio = ratio[mask]
        worst[f] = float(ratio.max()) if ratio.size else 0.0
    return worst


def rel_err_stats(gpu, ref, fields=FIELDS):
    """Max and RMS relative error per output (h, e against their magnitude sums), over the
    cells where the oracle's value is finite; a non-finite GPU value there counts as an
    infinite error (so a NaN from the kernel cannot drop out of the statistics)."""
    fields = [f for f in fields if f != "iters"]
    out = {}
    for f in fields:
        g, r = gpu[f], ref[f]
        scale = ref["h_scale"] if f == "h" else ref["e_scale"] if f == "e" else np.abs(r)
        ok = np.isfinite(r) & np.isfinite(scale) & (scale > 0)
        rel = np.where(np.isfinite(g), np.abs(g - r), np.inf)[ok] / scale[ok]
        out[f] = (float(rel.max()) if rel.size else float("nan"),
                  float(np.sqrt(np.mean(rel ** 2))) if rel.size else float("nan"))
    return out


# Chung's correlation coefficients a_i + b_i omega of E1..E4 (viscosity) and B1..B4
# (conductivity) for non-polar species (Chung et al. 1988), the part of the tables that
# sets the denominator E1 E4 + E2 + E3 of the density function G2.
CHUNG_E = np.array([[6.324, 50.412], [1.210e-3, -1.154e-3], [5.283, 254.209], [6.623, 38.096]])
CHUNG_B = np.array([[2.4166, 0.74824], [-0.50924, -1.5094], [6.6107, 5.6207], [14.543, -8.9139]])


def chung_kappa(species, Y):
    """Per-cell condition numbers of Chung's viscosity and conductivity (kappa_mu,
    kappa_lambda) from the denominator D = E1 E4 + E2 + E3 of the density function G2, which
    vanishes at one value of the pseudo-mixture acentric factor omega_m (about -0.067 for
    the viscosity set; H2, omega = -0.216, mixed with other species sweeps through it).

    Both outputs are proportional to 1/D in their dense part, so their relative rounding
    error is that of D: at most a few units of u times the sum of the magnitudes of what D
    is built from (E1 E4, E2, E3, the a_i and b_i omega_m inside each E_i) plus
    |dD/d omega| |omega_m| times the few roundings omega_m itself carries (a ratio of two
    sums: 4), divided by |D|.  omega_m = sum X_i omega_i p_i / sum X_i p_i with
    p_i = sigma_i^1.5, sigma_i = 0.809 Vc_i^(1/3) (Chung's one-fluid rules)."""
    W = np.array([s["W"] for s in species])
    X = (Y / W[:, None]) / (Y / W[:, None]).sum(0, keepdims=True)
    p = (0.809 * (np.array([s["Vc"] for s in species]) * 1e6) ** (1 / 3)) ** 1.5
    om = np.array([s["omega"] for s in species])
    wm = (X * (om * p)[:, None]).sum(0) / (X * p[:, None]).sum(0)
    out = []
    for C in (CHUNG_E, CHUNG_B):
        e = C[:, 0][:, None] + C[:, 1][:, None] * wm[None, :]
        D = e[0] * e[3] + e[1] + e[2]
        inner = np.abs(C[:, 0])[:, None] + np.abs(C[:, 1][:, None] * wm[None, :])
        mag = (np.abs(e[0] * e[3]) + np.abs(e[1]) + np.abs(e[2]) + inner[0] * np.abs(e[3]) + np.abs(e[0]) * inner[3]
               + inner[1] + inner[2])
        dD = C[0, 1] * e[3] + e[0] * C[3, 1] + C[1, 1] + C[2, 1]
        out.append(np.maximum(1.0, (mag + 4.0 * np.abs(dD * wm)) / np.abs(D)))
    return out[0], out[1]
