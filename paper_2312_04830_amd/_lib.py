"""ctypes binding of include/props.h (names and semantics follow the C ABI)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# PROPS_LIBRARY may name another build of the same library (e.g. a tuning variant)
library_path = os.environ.get("PROPS_LIBRARY", os.path.join(_HERE, "libprops.so"))

PTY, RHOEY, HPY = 0, 1, 2
FP64, MIXED = 0, 1
MAX_SPECIES = 8

status_bits = {
    "NONPHYS": 1, "NEWTON_MAXIT": 2, "BRACKET": 4, "THREE_ROOT": 8,
    "GIBBS_TIE": 16, "CV_NONPOS": 32, "OUT_OF_HULL": 64, "FALLBACK": 128,
}

ERR_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ETOOBIG",
             -5: "ETIMEDOUT", -6: "ENOTREADY"}


class PropsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class SpeciesDesc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("W", "Tc", "Pc", "Vc", "omega", "dipole", "kappa", "Tmid")] + \
               [("nasa_lo", ctypes.c_double * 7), ("nasa_hi", ctypes.c_double * 7)]


_P = ctypes.c_void_p


IN_FIELDS = ("P", "T", "rho", "e", "Y", "T_guess", "h")


class PropsIn(ctypes.Structure):
    _fields_ = [(n, _P) for n in IN_FIELDS]


OUT_FIELDS = ("T", "P", "Z", "rho", "h", "e", "cp", "c", "mu", "lambda")
EXTRA_OUT_FIELDS = ("psi", "alpha", "hRT")   # solver outputs; hRT is [ns][n]


class PropsOut(ctypes.Structure):
    _fields_ = [(n, _P) for n in OUT_FIELDS] + [("iters", _P)] + [(n, _P) for n in EXTRA_OUT_FIELDS]


class TrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("total_epochs", ctypes.c_int), ("batch", ctypes.c_int),
                ("lr", ctypes.c_float), ("lr_min", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("fit_scalers", ctypes.c_int)]


class TrainReport(ctypes.Structure):
    _fields_ = [("epochs_run", ctypes.c_int), ("steps", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("samples_per_s", ctypes.c_double), ("loss", ctypes.POINTER(ctypes.c_float))]


DNN_LAYERS = ((256, 10), (256, 256), (256, 256), (256, 256), (6, 256))
NIN, NOUT = 10, 6     # PROPS_DNN_IN, PROPS_DNN_OUT
DNN_NOALLOC_MAX_CELLS = 4194304   # PROPS_DNN_NOALLOC_MAX_CELLS

ROUTE_PR_FP64, ROUTE_PR_MIXED, ROUTE_DNN = 0, 1, 2
EXEC_GPU, EXEC_MOCK = 0, 1


class ServeCfg(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_int64), ("chunk_cells", ctypes.c_int64), ("max_inflight", ctypes.c_int),
                ("streams", ctypes.c_int), ("executor", ctypes.c_int), ("mock_ns_per_cell", ctypes.c_double),
                ("mock_species", ctypes.c_int)]


MEM_DEVICE, MEM_HOST = 0, 1


class Request(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("route", ctypes.c_int), ("n", ctypes.c_int64),
                ("inp", PropsIn), ("out", PropsOut), ("status", _P), ("memory", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("rc", ctypes.c_int), ("n", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("latency_s", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "failed", "queued_requests",
                                              "inflight_chunks", "cells_done", "slots", "slot_bytes")] + \
               [(k, ctypes.c_double) for k in ("elapsed_s", "cells_per_s", "p50_s", "p99_s", "mean_s", "max_s")]

_lib = None


def lib():
    """Load libprops.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise ImportError(f"{library_path} is missing: build it with "
                              "`python -m paper_2312_04830_amd.build`")
        L = ctypes.CDLL(library_path)
        L.props_last_error.restype = ctypes.c_char_p
        L.props_version.restype = ctypes.c_char_p
        L.props_mech_create.argtypes = [ctypes.POINTER(SpeciesDesc), ctypes.c_int, _P, ctypes.POINTER(_P)]
        L.props_mech_destroy.argtypes = [_P]
        L.props_mech_destroy.restype = None
        L.props_mech_num_species.argtypes = [_P]
        L.props_mech_set_newton.argtypes = [_P, ctypes.c_int, ctypes.c_double]
        L.props_pr.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(PropsIn),
                               ctypes.POINTER(PropsOut), ctypes.c_int64, _P, _P]
        L.props_diffusion.argtypes = [_P, ctypes.c_int, _P, _P, _P, _P, ctypes.c_int64, _P, _P]
        L.props_dnn_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(_P)]
        L.props_dnn_create_ex.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_P)]
        L.props_dnn_get_shape.argtypes = [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.props_dnn_destroy.argtypes = [_P]
        L.props_dnn_destroy.restype = None
        L.props_dnn_get_layer.argtypes = [_P, ctypes.c_int, _P, _P]
        L.props_dnn_set_layer.argtypes = [_P, ctypes.c_int, _P, _P]
        L.props_dnn_get_scalers.argtypes = [_P, _P, _P, _P, _P]
        L.props_dnn_set_scalers.argtypes = [_P, _P, _P, _P, _P]
        L.props_dnn_set_log_outputs.argtypes = [_P, ctypes.c_uint]
        L.props_dnn_get_log_outputs.argtypes = [_P, ctypes.POINTER(ctypes.c_uint)]
        L.props_dnn_save.argtypes = [_P, ctypes.c_char_p]
        L.props_dnn_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(_P)]
        L.props_dnn.argtypes = [_P, _P, ctypes.POINTER(PropsIn), ctypes.POINTER(PropsOut),
                                ctypes.c_int64, _P, _P]
        L.props_dnn_noalloc.argtypes = [_P, _P, ctypes.POINTER(PropsIn), ctypes.POINTER(PropsOut),
                                        ctypes.c_int64, _P, _P]
        L.props_dnn_grad.argtypes = [_P, _P, _P, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_float), _P]
        L.props_dnn_features.argtypes = [_P, _P, _P, ctypes.c_int64, _P]
        L.props_stream_copy.argtypes = [_P, _P, ctypes.c_size_t, _P]
        L.props_features_hpz.argtypes = [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         _P, _P, _P, ctypes.c_int64, _P, _P]
        L.train_dnn.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.POINTER(TrainCfg),
                                ctypes.POINTER(TrainReport), _P]
        L.serve_create.argtypes = [ctypes.POINTER(ServeCfg), _P, _P, ctypes.POINTER(_P)]
        L.serve_submit.argtypes = [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.serve_wait.argtypes = [_P, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(Result)]
        L.serve_stats.argtypes = [_P, ctypes.POINTER(ServeStats)]
        L.serve_destroy.argtypes = [_P]
        L.serve_destroy.restype = None
        _lib = L
    return _lib


def check(rc):
    if rc < 0:
        raise PropsError(rc, lib().props_last_error().decode())
    return rc


def _ptr(t):
    """Device pointer of a tensor (None -> NULL); requires contiguous storage."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to libprops must be contiguous")
    return t.data_ptr()


def _arg(t, count, dtype, name):
    """Device pointer of a tensor the library will read or write `count` elements of: the
    tensor must be a contiguous CUDA tensor of `dtype` with at least `count` elements (a
    short, host or mistyped array would otherwise be read or written out of bounds on the
    device).  None -> NULL."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: expected a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if t.numel() < count:
        raise ValueError(f"{name}: {t.numel()} elements, the call needs {count}")
    return _ptr(t)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Mechanism:
    """props_mech_create on the current device from species dicts (SI units)."""

    def __init__(self, species, kij=None):
        ns = len(species)
        arr = (SpeciesDesc * ns)()
        for i, s in enumerate(species):
            d = arr[i]
            for k in ("W", "Tc", "Pc", "Vc", "omega", "dipole", "kappa", "Tmid"):
                setattr(d, k, float(s[k]))
            for k in range(7):
                d.nasa_lo[k] = float(s["nasa_lo"][k])
                d.nasa_hi[k] = float(s["nasa_hi"][k])
        kbuf = None
        if kij is not None:
            flat = [float(x) for row in kij for x in row]
            kbuf = (ctypes.c_double * len(flat))(*flat)
        h = _P()
        check(lib().props_mech_create(arr, ns, ctypes.cast(kbuf, _P) if kbuf is not None else None,
                                      ctypes.byref(h)))
        self.handle = h
        self.ns = ns

    def set_newton(self, max_iter=100, rtol=1e-10):
        check(lib().props_mech_set_newton(self.handle, int(max_iter), float(rtol)))

    def close(self):
        if getattr(self, "handle", None):
            lib().props_mech_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pr(mech, mode, prec, inputs, outputs, n, status=None, stream=None):
    """props_pr: ``inputs``/``outputs`` map C field names to contiguous float64 device
    tensors (missing or None = NULL); Y and hRT hold [ns, n], iters and status uint8 [n]."""
    import torch
    n = int(n)
    size = lambda k: mech.ns * n if k in ("Y", "hRT") else n  # noqa: E731
    pin = PropsIn(**{k: _arg(inputs.get(k), size(k), torch.float64, k) for k in IN_FIELDS})
    pout = PropsOut(**{k: _arg(outputs.get(k), size(k), torch.uint8 if k == "iters" else torch.float64, k)
                       for k in OUT_FIELDS + ("iters",) + EXTRA_OUT_FIELDS})
    check(lib().props_pr(mech.handle, int(mode), int(prec), ctypes.byref(pin), ctypes.byref(pout),
                         n, _arg(status, n, torch.uint8, "status"), _stream(stream)))


def diffusion(mech, prec, P, T, Y, D, n, status=None, stream=None):
    """props_diffusion: P, T [n], Y and D [ns, n] are contiguous float64 device tensors."""
    import torch
    n, f8 = int(n), torch.float64
    m = mech.ns * n
    check(lib().props_diffusion(mech.handle, int(prec), _arg(P, n, f8, "P"), _arg(T, n, f8, "T"),
                                _arg(Y, m, f8, "Y"), _arg(D, m, f8, "D"), n,
                                _arg(status, n, torch.uint8, "status"), _stream(stream)))


def features_hpz(species, fuel, oxidizer, bc_lambda, h, P, Y, n, X, stream=None):
    """props_features_hpz: species dicts give W and "atoms" {C, H, O}; h, P [n], Y [ns, n]
    and X [10, n] are float64 device tensors."""
    import numpy as np
    import torch
    atoms = np.ascontiguousarray([[s["atoms"][e] for e in ("C", "H", "O")] for s in species], dtype=np.int32)
    W = np.ascontiguousarray([s["W"] for s in species], dtype=np.float64)
    n, f8 = int(n), torch.float64
    check(lib().props_features_hpz(atoms.ctypes.data, W.ctypes.data, len(species), int(fuel), int(oxidizer),
                                   float(bc_lambda), _arg(h, n, f8, "h"), _arg(P, n, f8, "P"),
                                   _arg(Y, len(species) * n, f8, "Y"), n, _arg(X, 10 * n, f8, "X"),
                                   _stream(stream)))


def stream_copy(src, dst, nbytes, stream=None):
    """props_stream_copy: device-to-device streaming copy of nbytes (the measured bandwidth
    ceiling); src and dst are device tensors."""
    check(lib().props_stream_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)))


def dnn_layers(hidden_layers=4, outputs=NOUT):
    """(out, in) of each weight layer of a network of that shape."""
    return ((256, NIN),) + ((256, 256),) * (hidden_layers - 1) + ((outputs, 256),)


class Network:
    """props_dnn_* handle: the MLP surrogate (10 -> hidden_layers x 256 GELU -> outputs;
    4 and 6 by default, the paper's networks have 3 hidden layers)."""

    def __init__(self, seed=0, handle=None, hidden_layers=4, outputs=NOUT):
        if handle is None:
            handle = _P()
            check(lib().props_dnn_create_ex(int(seed), int(hidden_layers), int(outputs), ctypes.byref(handle)))
        self.handle = handle
        nh, no = ctypes.c_int(), ctypes.c_int()
        check(lib().props_dnn_get_shape(self.handle, ctypes.byref(nh), ctypes.byref(no)))
        self.hidden_layers, self.outputs = nh.value, no.value
        self.layers = dnn_layers(self.hidden_layers, self.outputs)

    @classmethod
    def load(cls, path):
        h = _P()
        check(lib().props_dnn_load(str(path).encode(), ctypes.byref(h)))
        return cls(handle=h)

    def save(self, path):
        check(lib().props_dnn_save(self.handle, str(path).encode()))

    def get_layer(self, l):
        import numpy as np
        o, i = self.layers[l]
        W = np.zeros((o, i), dtype=np.float32)
        b = np.zeros(o, dtype=np.float32)
        check(lib().props_dnn_get_layer(self.handle, l, W.ctypes.data, b.ctypes.data))
        return W, b

    def set_layer(self, l, W, b):
        import numpy as np
        W = np.ascontiguousarray(W, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        assert W.shape == self.layers[l] and b.shape == (self.layers[l][0],)
        check(lib().props_dnn_set_layer(self.handle, l, W.ctypes.data, b.ctypes.data))

    def get_scalers(self):
        import numpy as np
        a = [np.zeros(k) for k in (10, 10, 6, 6)]
        check(lib().props_dnn_get_scalers(self.handle, *[x.ctypes.data for x in a]))
        return a

    def set_scalers(self, in_lo, in_hi, out_lo, out_hi):
        import numpy as np
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (in_lo, in_hi, out_lo, out_hi)]
        check(lib().props_dnn_set_scalers(self.handle, *[x.ctypes.data for x in a]))

    def set_log_outputs(self, mask):
        """Bit j: output j is trained on and predicted as its logarithm (before train)."""
        check(lib().props_dnn_set_log_outputs(self.handle, int(mask)))

    def get_log_outputs(self):
        m = ctypes.c_uint()
        check(lib().props_dnn_get_log_outputs(self.handle, ctypes.byref(m)))
        return m.value

    def _dnn_args(self, inputs, outputs, n, status):
        import torch
        ns = NIN - 2
        pin = PropsIn(**{k: _arg(inputs.get(k), ns * n if k == "Y" else n, torch.float64, k) for k in IN_FIELDS})
        pout = PropsOut(**{k: _arg(outputs.get(k), n, torch.uint8 if k == "iters" else torch.float64, k)
                           for k in OUT_FIELDS + ("iters",)})
        return pin, pout, _arg(status, n, torch.uint8, "status")

    def __call__(self, inputs, outputs, n, fallback=None, status=None, stream=None):
        """props_dnn: inputs P, T, Y [8, n]; outputs rho, h, cp, c, mu, lambda (float64 device
        tensors); status uint8 [n]."""
        n = int(n)
        pin, pout, st = self._dnn_args(inputs, outputs, n, status)
        check(lib().props_dnn(self.handle, fallback.handle if fallback is not None else None,
                              ctypes.byref(pin), ctypes.byref(pout), n, st, _stream(stream)))

    def noalloc(self, inputs, outputs, n, fallback=None, status=None, stream=None):
        """props_dnn_noalloc: props_dnn with its fallback list in the library's static device
        array (allocates nothing; n <= DNN_NOALLOC_MAX_CELLS; calls on one device must not
        overlap)."""
        n = int(n)
        pin, pout, st = self._dnn_args(inputs, outputs, n, status)
        check(lib().props_dnn_noalloc(self.handle, fallback.handle if fallback is not None else None,
                                      ctypes.byref(pin), ctypes.byref(pout), n, st, _stream(stream)))

    def features(self, X, Y, n, stream=None):
        """props_dnn_features: X [10, n] raw features, Y [6, n] outputs (float64 device tensors)."""
        import torch
        n = int(n)
        check(lib().props_dnn_features(self.handle, _arg(X, NIN * n, torch.float64, "X"),
                                       _arg(Y, self.outputs * n, torch.float64, "Y"), n, _stream(stream)))

    def grad(self, X, Y, n, stream=None):
        """props_dnn_grad on device X [10, n], Y [6, n] (float32): (loss, flat gradient)."""
        import numpy as np
        total = sum(o * i + o for o, i in self.layers)
        g = np.zeros(total, dtype=np.float32)
        loss = ctypes.c_float()
        import torch
        n = int(n)
        check(lib().props_dnn_grad(self.handle, _arg(X, NIN * n, torch.float32, "X"),
                                   _arg(Y, self.outputs * n, torch.float32, "Y"), n, g.ctypes.data,
                                   ctypes.byref(loss), _stream(stream)))
        return loss.value, g

    def train(self, X, Y, n, epochs, batch=65536, lr=1e-3, lr_min=1e-5, total_epochs=0,
              seed=0, fit_scalers=True, stream=None):
        """train_dnn on device X [10, n], Y [6, n]; returns (report dict, per-epoch losses)."""
        import numpy as np
        cfg = TrainCfg(epochs=int(epochs), total_epochs=int(total_epochs), batch=int(batch), lr=lr,
                       lr_min=lr_min, beta1=0.9, beta2=0.999, eps=1e-8, seed=int(seed),
                       fit_scalers=int(bool(fit_scalers)))
        losses = np.zeros(max(1, int(epochs)), dtype=np.float32)
        rep = TrainReport(loss=losses.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        import torch
        n = int(n)
        check(lib().train_dnn(self.handle, _arg(X, NIN * n, torch.float32, "X"),
                              _arg(Y, self.outputs * n, torch.float32, "Y"), n, ctypes.byref(cfg),
                              ctypes.byref(rep), _stream(stream)))
        return {"epochs": rep.epochs_run, "steps": rep.steps, "seconds": rep.seconds,
                "samples_per_s": rep.samples_per_s}, losses[:int(epochs)]

    def close(self):
        if getattr(self, "handle", None):
            lib().props_dnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_ptr(a, count=0, itemsize=8, name="array"):
    """Address of a host array (numpy or CPU tensor) the server will read or write `count`
    elements of (`itemsize` bytes each: float64, or uint8 for status); None -> NULL."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        if a.is_cuda or not a.is_contiguous():
            raise ValueError("serving requests take contiguous host arrays")
        size, isz, ptr = a.numel(), a.element_size(), a.data_ptr()
    else:
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("serving requests take contiguous host arrays")
        size, isz, ptr = a.size, a.itemsize, a.ctypes.data
    if isz != itemsize or size < count:
        raise ValueError(f"{name}: needs {count} elements of {itemsize} bytes, got {size} of {isz}")
    return ptr


class Server:
    """serve_*: chunked, memory-admitted, multi-stream property server."""

    def __init__(self, mech, dnn=None, mem_budget=1 << 30, chunk_cells=262144, max_inflight=0,
                 streams=4, executor=EXEC_GPU, mock_ns_per_cell=0.0, mock_species=8):
        cfg = ServeCfg(mem_budget=int(mem_budget), chunk_cells=int(chunk_cells), max_inflight=int(max_inflight),
                       streams=int(streams), executor=int(executor), mock_ns_per_cell=float(mock_ns_per_cell),
                       mock_species=int(mock_species))
        h = _P()
        check(lib().serve_create(ctypes.byref(cfg), mech.handle if mech is not None else None,
                                 dnn.handle if dnn is not None else None, ctypes.byref(h)))
        self.handle = h
        self.ns = mech.ns if mech is not None else int(mock_species)
        self._keep = {}

    def submit(self, mode, route, n, inputs, outputs, status=None):
        """Non-blocking.  Arrays are either all device tensors (a device-resident request,
        evaluated in place; the inputs must be ready, e.g. after a synchronize) or all numpy
        host arrays (staged through the server's slots); they must stay alive until wait()
        returns."""
        import torch
        n = int(n)
        arrays = [a for a in list(inputs.values()) + list(outputs.values()) + [status] if a is not None]
        on_dev = [isinstance(a, torch.Tensor) and a.is_cuda for a in arrays]
        if any(on_dev) and not all(on_dev):
            raise ValueError("serve request: mix of device tensors and host arrays")
        size = lambda k: self.ns * n if k in ("Y", "hRT") else n  # noqa: E731
        if arrays and all(on_dev):
            f8, u8 = torch.float64, torch.uint8
            req = Request(mode=int(mode), route=int(route), n=n, memory=MEM_DEVICE,
                          inp=PropsIn(**{k: _arg(inputs.get(k), size(k), f8, k) for k in IN_FIELDS}),
                          out=PropsOut(**{k: _arg(outputs.get(k), size(k), u8 if k == "iters" else f8, k)
                                          for k in OUT_FIELDS + ("iters",) + EXTRA_OUT_FIELDS}),
                          status=_arg(status, n, u8, "status"))
        else:
            req = Request(mode=int(mode), route=int(route), n=n, memory=MEM_HOST,
                          inp=PropsIn(**{k: _host_ptr(inputs.get(k), size(k), 8, k) for k in IN_FIELDS}),
                          out=PropsOut(**{k: _host_ptr(outputs.get(k), size(k), 1 if k == "iters" else 8, k)
                                          for k in OUT_FIELDS + ("iters",) + EXTRA_OUT_FIELDS}),
                          status=_host_ptr(status, n, 1, "status"))
        t = ctypes.c_uint64()
        check(lib().serve_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (inputs, outputs, status)
        return t.value

    def wait(self, ticket, timeout_us=-1):
        res = Result()
        rc = lib().serve_wait(self.handle, int(ticket), int(timeout_us), ctypes.byref(res))
        if rc != -5:   # not a time-out: the ticket is retired
            self._keep.pop(ticket, None)
        check(rc)
        return {"rc": res.rc, "n": res.n, "t_submit": res.t_submit, "t_done": res.t_done, "latency_s": res.latency_s}

    def stats(self):
        st = ServeStats()
        check(lib().serve_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServeStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().serve_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
