"""props_dnn_noalloc, the surrogate entry point that allocates nothing (its fallback list
lives in the library's static device array), against props_dnn: the same outputs and
status, bit for bit, on two calls in a row, the second with fewer cells, with cells outside
the training box recomputed by the PR fallback."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KEYS = ("rho", "h", "cp", "c", "mu", "lambda")


@pytest.fixture(scope="module")
def props():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_04830_amd as P
    P.lib()
    return P


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def trained_box_network(props):
    """A network whose input box is that of (P, T, Y) training states, so that the hot and
    high-pressure cells planted below fall outside it."""
    P, T, Y = synth.training_states(20_000, seed=71)
    X = np.vstack([P, T, Y])
    net = props.Network(seed=12)
    olo = np.array([0.0, -1e7, 5.0, 100.0, -13.0, -5.0])
    ohi = np.array([7.0, 1e7, 12.0, 2000.0, -7.0, 1.0])
    net.set_scalers(X.min(1), X.max(1), olo, ohi)
    return net


def field(n, seed):
    res = int(np.ceil(n ** (1 / 3)))
    P, T, Y = synth.flame_field(res, seed=seed)
    P, T, Y = P[:n].copy(), T[:n].copy(), np.ascontiguousarray(Y[:, :n])
    T[::9] = 3400.0          # above the training box
    P[::13] = 2.2e7          # above the training box
    Y[:, 5] = 0.0            # sum Y = 0: non-physical
    return P, T, Y


def run(props, net, mech, P, T, Y, noalloc):
    import torch
    n = T.size
    ins = {"P": dev(P), "T": dev(T), "Y": dev(Y)}
    outs = {k: torch.full((n,), -1.0, dtype=torch.float64, device="cuda:0") for k in KEYS}
    st = torch.full((n,), 3, dtype=torch.uint8, device="cuda:0")
    (net.noalloc if noalloc else net)(ins, outs, n, fallback=mech, status=st)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in outs.items()}, st.cpu().numpy()


def test_noalloc_matches_props_dnn_on_two_calls(props):
    mech = props.Mechanism(synth.load_species(synth.FLAME_SPECIES), synth.synthetic_kij(8))
    net = trained_box_network(props)
    for n, seed in ((300_001, 21), (70_001, 22)):    # the second call is smaller
        print(f"[no-alloc] n = {n}, seed {seed}", flush=True)
        P, T, Y = field(n, seed)
        o_ref, s_ref = run(props, net, mech, P, T, Y, noalloc=False)
        o_new, s_new = run(props, net, mech, P, T, Y, noalloc=True)
        fb = (s_ref & 128) != 0
        assert fb.sum() >= n // 9 and not fb.all()        # the fallback really ran
        assert np.array_equal(s_new, s_ref)
        for k in KEYS:
            assert np.array_equal(o_new[k].view(np.int64), o_ref[k].view(np.int64)), k


def test_noalloc_refuses_more_cells_than_its_list(props):
    import torch
    mech = props.Mechanism(synth.load_species(synth.FLAME_SPECIES))
    net = props.Network(seed=1)
    tiny = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    p = tiny.data_ptr()
    pin = props._lib.PropsIn(P=p, T=p, Y=p)
    pout = props._lib.PropsOut(rho=p)
    rc = props.lib().props_dnn_noalloc(net.handle, mech.handle, ctypes.byref(pin), ctypes.byref(pout),
                                       props._lib.DNN_NOALLOC_MAX_CELLS + 1, None, None)
    assert rc == -4, props.lib().props_last_error()       # PROPS_ETOOBIG, nothing launched
    assert b"static fallback list" in props.lib().props_last_error()
