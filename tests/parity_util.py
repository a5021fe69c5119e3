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


def compare(gpu, ref, mode, rtol, fields=FIELDS, mask=None, kappa=True):
    """Return {field: worst err/tol}; h and e are compared against their sums of
    magnitudes (they cross zero), everything else relative to itself."""
    k = cell_kappa(ref, mode) if kappa else np.ones(len(ref))
    worst = {}
    for f in fields:
        g = gpu[f]
        r = ref["lambda"] if f == "lambda" else ref[f]
        if f == "h":
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
    """Max and RMS relative error per output (h, e against their magnitude sums)."""
    fields = [f for f in fields if f != "iters"]
    out = {}
    for f in fields:
        g, r = gpu[f], ref[f]
        scale = ref["h_scale"] if f == "h" else ref["e_scale"] if f == "e" else np.abs(r)
        rel = np.abs(g - r) / scale
        ok = np.isfinite(rel)
        out[f] = (float(rel[ok].max()) if ok.any() else float("nan"),
                  float(np.sqrt(np.mean(rel[ok] ** 2))) if ok.any() else float("nan"))
    return out
