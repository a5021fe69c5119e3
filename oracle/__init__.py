"""CPU oracle for the real-fluid property path — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package.  It is independent of the GPU library: it builds its own C source
(``pr_oracle.c``) with gcc, parses species dictionaries itself and shares no code,
header, table or constant with the product path.

``build()`` compiles ``liboracle.so`` next to this file; ``Mech`` wraps a mechanism;
``Mech.eval`` runs the oracle over a batch of cells and returns a numpy structured array
with one record per cell (fields as in ``orc_cell`` of the C source).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a test of the tests may point the loader at a deliberately broken build
_LIB_LOAD = os.environ.get("ORACLE_LIB_OVERRIDE", _LIB)
MAXNS = 16

PT, RHOE, VT, HP = 0, 1, 2, 3
NONPHYS, NEWTON_MAXIT, BRACKET, THREE_ROOT, GIBBS_TIE, CV_NONPOS = 1, 2, 4, 8, 16, 32


def build(force=True):
    """Compile the oracle (gcc -O2, no fast-math, OpenMP over cells)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Species(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("W", "Tc", "Pc", "Vc", "omega", "dipole", "kappa", "Tmid")] + \
               [("lo", ctypes.c_double * 7), ("hi", ctypes.c_double * 7)]


class _Mech(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("pad", ctypes.c_int),
                ("sp", _Species * MAXNS), ("kij", ctypes.c_double * (MAXNS * MAXNS))]


CELL_DTYPE = np.dtype([(n, "f8") for n in (
    "T", "P", "Z", "rho", "v", "W", "h", "e", "cp", "cv", "c", "mu", "lambda",
    "am", "dam", "d2am", "bm", "A", "B", "h_ig", "e_ig", "cp_ig", "cv_ig",
    "h_scale", "e_scale", "kappa_Z", "kappa_cp", "kappa_T", "psi", "alpha", "mu_scale", "lambda_scale")] +
    [("hRT", "f8", (MAXNS,)), ("roots", "f8", (3,)), ("nroots", "i4"), ("nphys", "i4"), ("status", "i4"), ("iters", "i4")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB_LOAD)
        L.orc_eval.restype = ctypes.c_int
        L.orc_eval.argtypes = [ctypes.POINTER(_Mech), ctypes.c_int, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        L.orc_cubic_roots.restype = ctypes.c_int
        L.orc_cubic_roots.argtypes = [ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)]
        L.orc_gdep_RT.restype = ctypes.c_double
        L.orc_gdep_RT.argtypes = [ctypes.c_double] * 3
        L.orc_mix.restype = None
        L.orc_mix.argtypes = [ctypes.POINTER(_Mech), ctypes.c_void_p, ctypes.c_double] + \
            [ctypes.POINTER(ctypes.c_double)] * 4
        for fn in ("orc_chung_mu",):
            getattr(L, fn).restype = ctypes.c_double
            getattr(L, fn).argtypes = [ctypes.c_double] * 8
        L.orc_chung_mu0.restype = ctypes.c_double
        L.orc_chung_mu0.argtypes = [ctypes.c_double] * 7
        L.orc_chung_lambda.restype = ctypes.c_double
        L.orc_chung_lambda.argtypes = [ctypes.c_double] * 9
        L.orc_omega_v.restype = ctypes.c_double
        L.orc_omega_v.argtypes = [ctypes.c_double]
        L.orc_pr_kappa.restype = ctypes.c_double
        L.orc_pr_kappa.argtypes = [ctypes.c_double]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_omega_d.restype = ctypes.c_double
        L.orc_omega_d.argtypes = [ctypes.c_double]
        L.orc_binary_diffusion.restype = ctypes.c_double
        L.orc_binary_diffusion.argtypes = [ctypes.c_double] * 6
        L.orc_eval_mixdiff.restype = ctypes.c_int
        L.orc_eval_mixdiff.argtypes = [ctypes.POINTER(_Mech), ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        assert L.orc_sizeof_cell() == CELL_DTYPE.itemsize, "orc_cell layout mismatch"
        assert L.orc_sizeof_mech() == ctypes.sizeof(_Mech), "orc_mech layout mismatch"
        _lib = L
    return _lib


class Mech:
    """A mechanism: species dictionaries (SI units) plus an optional k_ij matrix."""

    def __init__(self, species, kij=None):
        ns = len(species)
        if not 1 <= ns <= MAXNS:
            raise ValueError("1..16 species supported")
        m = _Mech()
        m.ns = ns
        for i, s in enumerate(species):
            sp = m.sp[i]
            for k in ("W", "Tc", "Pc", "Vc", "omega", "dipole", "kappa", "Tmid"):
                setattr(sp, k, float(s[k]))
            for k in range(7):
                sp.lo[k] = float(s["nasa_lo"][k])
                sp.hi[k] = float(s["nasa_hi"][k])
        if kij is not None:
            kij = np.asarray(kij, dtype=np.float64).reshape(ns, ns)
            for i in range(ns):
                for j in range(ns):
                    m.kij[i * ns + j] = kij[i, j]
        self.ns = ns
        self.species = species
        self._m = m

    def eval(self, mode, in0, in1, Y, transport=True, nthreads=0):
        """Run the oracle on n cells; Y is [ns, n]. Returns a CELL_DTYPE array."""
        in0 = np.ascontiguousarray(in0, dtype=np.float64).ravel()
        in1 = np.ascontiguousarray(in1, dtype=np.float64).ravel()
        n = in0.size
        Y = np.ascontiguousarray(np.asarray(Y, dtype=np.float64).reshape(self.ns, n))
        out = np.zeros(n, dtype=CELL_DTYPE)
        rc = lib().orc_eval(ctypes.byref(self._m), int(mode), n, in0.ctypes.data,
                            in1.ctypes.data, Y.ctypes.data, int(bool(transport)),
                            out.ctypes.data, int(nthreads))
        if rc != 0:
            raise RuntimeError("orc_eval failed")
        return out

    def state_PT(self, P, T, Y, **kw):
        return self.eval(PT, P, T, Y, **kw)

    def state_rhoe(self, rho, e, Y, **kw):
        return self.eval(RHOE, rho, e, Y, **kw)

    def state_vT(self, v, T, Y, **kw):
        return self.eval(VT, v, T, Y, **kw)

    def state_hP(self, h, P, Y, **kw):
        return self.eval(HP, h, P, Y, **kw)

    def mixdiff(self, P, T, Y, nthreads=0):
        """Mixture-averaged diffusion coefficients [ns, n] (m^2/s) at (P, T, Y)."""
        P = np.ascontiguousarray(P, dtype=np.float64).ravel()
        T = np.ascontiguousarray(T, dtype=np.float64).ravel()
        n = P.size
        Y = np.ascontiguousarray(np.asarray(Y, dtype=np.float64).reshape(self.ns, n))
        D = np.zeros((self.ns, n))
        if lib().orc_eval_mixdiff(ctypes.byref(self._m), n, P.ctypes.data, T.ctypes.data, Y.ctypes.data,
                                  D.ctypes.data, int(nthreads)) != 0:
            raise RuntimeError("orc_eval_mixdiff failed")
        return D

    def mix(self, X, T):
        X = np.ascontiguousarray(X, dtype=np.float64)
        out = [ctypes.c_double() for _ in range(4)]
        lib().orc_mix(ctypes.byref(self._m), X.ctypes.data, float(T), *[ctypes.byref(o) for o in out])
        return tuple(o.value for o in out)


def cubic_roots(A, B):
    buf = (ctypes.c_double * 3)()
    k = lib().orc_cubic_roots(float(A), float(B), buf)
    return [buf[i] for i in range(k)]


def gdep_RT(Z, A, B):
    return lib().orc_gdep_RT(float(Z), float(A), float(B))


def chung_mu(T, rho_molar, Tc, Vc_cm3, M_gmol, omega, mu_r=0.0, kappa=0.0):
    return lib().orc_chung_mu(T, rho_molar, Tc, Vc_cm3, M_gmol, omega, mu_r, kappa)


def chung_mu0(T, Tc, Vc_cm3, M_gmol, omega, mu_r=0.0, kappa=0.0):
    return lib().orc_chung_mu0(T, Tc, Vc_cm3, M_gmol, omega, mu_r, kappa)


def chung_lambda(T, rho_molar, Tc, Vc_cm3, M_gmol, omega, mu_r, kappa, Cv):
    return lib().orc_chung_lambda(T, rho_molar, Tc, Vc_cm3, M_gmol, omega, mu_r, kappa, Cv)


def omega_v(Ts):
    return lib().orc_omega_v(Ts)


def omega_d(Ts):
    return lib().orc_omega_d(Ts)


def binary_diffusion(T, P, Mi, Mj, sigma, eps_k):
    return lib().orc_binary_diffusion(T, P, Mi, Mj, sigma, eps_k)


def max_threads():
    return lib().orc_max_threads()
