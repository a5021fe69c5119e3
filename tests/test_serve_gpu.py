"""The property server on the GPU: results equal the direct library calls bit for bit, and a
request's result is the same alone and in a mix of concurrent requests."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KEYS6 = ("rho", "h", "cp", "c", "mu", "lambda")
KEYS10 = ("T", "P", "Z", "rho", "h", "e", "cp", "c", "mu", "lambda")


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_04830_amd as P
    sp = synth.load_species(synth.FLAME_SPECIES)
    mech = P.Mechanism(sp, synth.synthetic_kij(8))
    net = P.Network(seed=4)
    Pf, Tf, Yf = synth.flame_field(16, seed=3)
    lo = np.array([Pf.min(), Tf.min()] + list(Yf.min(1)))
    hi = np.array([Pf.max(), Tf.max()] + list(Yf.max(1)))
    net.set_scalers(lo, hi, np.array([2.0, -1e7, 7.0, 200.0, -11.5, -3.9]),
                    np.array([7.0, 2e6, 9.5, 1500.0, -8.0, -1.0]))
    return P, mech, net


def req(n, seed, res=12):
    P_, T_, Y_ = synth.flame_field(res, seed=seed)
    k = np.random.default_rng(seed).integers(0, T_.size - n) if T_.size > n else 0
    sl = slice(k, k + n)
    return {"P": P_[sl].copy(), "T": T_[sl].copy(), "Y": np.ascontiguousarray(Y_[:, sl])}


def outputs(n, keys):
    return {k: np.full(n, np.nan) for k in keys}


def run_alone(P, server, mode, route, ins, keys):
    n = ins["Y"].shape[1]
    o = outputs(n, keys)
    st = np.zeros(n, dtype=np.uint8)
    server.wait(server.submit(mode, route, n, ins, o, st))
    return o, st


def rhoe_inputs(P, mech, ins):
    import torch
    n = ins["Y"].shape[1]
    d = {k: torch.from_numpy(v).to("cuda:0") for k, v in ins.items()}
    rho = torch.empty(n, dtype=torch.float64, device="cuda:0")
    e = torch.empty_like(rho)
    P.pr(mech, P.PTY, P.FP64, d, {"rho": rho, "e": e}, n)
    torch.cuda.synchronize()
    return {"rho": rho.cpu().numpy(), "e": e.cpu().numpy(), "Y": ins["Y"], "T_guess": ins["T"] * 1.003}


def test_server_equals_direct_calls(env):
    import torch
    P, mech, net = env
    s = P.Server(mech, net, mem_budget=256 << 20, chunk_cells=4096, streams=3)
    ins = req(1500, 1, res=14)
    n = 1500
    d = {k: torch.from_numpy(v).to("cuda:0") for k, v in ins.items()}
    for route, prec in ((P.ROUTE_PR_FP64, P.FP64), (P.ROUTE_PR_MIXED, P.MIXED)):
        o, st = run_alone(P, s, P.PTY, route, ins, KEYS10)
        od = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in KEYS10}
        sd = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        P.pr(mech, P.PTY, prec, d, od, n, status=sd)
        torch.cuda.synchronize()
        for k in KEYS10:
            assert np.array_equal(o[k], od[k].cpu().numpy(), equal_nan=True), (route, k)
        assert np.array_equal(st, sd.cpu().numpy())
    o, st = run_alone(P, s, P.PTY, P.ROUTE_DNN, ins, KEYS6)
    od = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in KEYS6}
    sd = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    net(d, od, n, fallback=mech, status=sd)
    torch.cuda.synchronize()
    for k in KEYS6:
        assert np.array_equal(o[k], od[k].cpu().numpy(), equal_nan=True), k
    assert np.array_equal(st, sd.cpu().numpy())
    s.close()


def test_alone_equals_in_the_mix(env):
    P, mech, net = env
    s = P.Server(mech, net, mem_budget=128 << 20, chunk_cells=2048, streams=4)
    base = req(5000, 7, res=20)
    cases = [(P.PTY, P.ROUTE_PR_MIXED, base, KEYS10), (P.PTY, P.ROUTE_DNN, base, KEYS6),
             (P.RHOEY, P.ROUTE_PR_FP64, rhoe_inputs(P, mech, base), KEYS10)]
    alone = [run_alone(P, s, m, r, i, k) for m, r, i, k in cases]
    # the same requests again, interleaved with 24 others of uneven sizes and routes
    rng = np.random.default_rng(3)
    mix = []
    for j in range(24):
        n = int(rng.integers(1, 9000))
        ins = req(min(n, 5000), 100 + j, res=18)
        route = [P.ROUTE_PR_MIXED, P.ROUTE_DNN, P.ROUTE_PR_FP64][j % 3]
        o = outputs(ins["Y"].shape[1], KEYS6)
        mix.append((s.submit(P.PTY, route, ins["Y"].shape[1], ins, o), o))
        if j == 5 or j == 15:
            for m, r, i, k in cases:
                o2 = outputs(i["Y"].shape[1], k)
                st2 = np.zeros(i["Y"].shape[1], dtype=np.uint8)
                mix.append((s.submit(m, r, i["Y"].shape[1], i, o2, st2), (o2, st2, len(mix))))
    results = []
    for t, o in mix:
        s.wait(t)
        if isinstance(o, tuple):
            results.append(o[:2])
    assert len(results) == 6
    for j, (o2, st2) in enumerate(results):
        o1, st1 = alone[j % 3]
        for k in o1:
            assert np.array_equal(o1[k].view(np.int64), o2[k].view(np.int64)), (j, k)
        assert np.array_equal(st1, st2)
    st = s.stats()
    assert st["failed"] == 0 and st["completed"] == 3 + len(mix)
    s.close()


def test_small_budget_still_completes(env):
    P, mech, net = env
    s = P.Server(mech, None, mem_budget=2 * 1024 * 1024, chunk_cells=4096, streams=2)
    assert s.stats()["slots"] >= 1
    ins = req(5000, 11, res=20)
    o, st = run_alone(P, s, P.PTY, P.ROUTE_PR_MIXED, ins, KEYS6)
    assert np.all(np.isfinite(o["rho"])) and np.all(st == 0)
    s.close()


def test_server_hpy_equals_direct_calls(env):
    """(h, P, Y) requests through the server equal a direct props_pr call bit for bit."""
    import torch
    P, mech, net = env
    s = P.Server(mech, net, mem_budget=256 << 20, chunk_cells=1024, streams=2)
    ins = req(3000, 11, res=16)
    n = 3000
    d = {k: torch.from_numpy(v).to("cuda:0") for k, v in ins.items()}
    h = torch.empty(n, dtype=torch.float64, device="cuda:0")
    P.pr(mech, P.PTY, P.FP64, d, {"h": h}, n)
    torch.cuda.synchronize()
    hin = {"h": h.cpu().numpy(), "P": ins["P"], "Y": ins["Y"], "T_guess": ins["T"] * 0.995}
    dh = {k: torch.from_numpy(v).to("cuda:0") for k, v in hin.items()}
    for route, prec in ((P.ROUTE_PR_FP64, P.FP64), (P.ROUTE_PR_MIXED, P.MIXED)):
        o, st = run_alone(P, s, P.HPY, route, hin, KEYS10)
        od = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in KEYS10}
        sd = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        P.pr(mech, P.HPY, prec, dh, od, n, status=sd)
        torch.cuda.synchronize()
        for k in KEYS10:
            assert np.array_equal(o[k], od[k].cpu().numpy(), equal_nan=True), (route, k)
        assert np.array_equal(st, sd.cpu().numpy())
        assert np.all(st == 0)
    s.close()


# ------------------------------------------------------------------ device-resident requests

def to_dev(d):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0") for k, v in d.items()}


def dev_outputs(n, keys, ns=8):
    import torch
    return {k: torch.full((ns, n) if k == "hRT" else (n,), float("nan"), dtype=torch.float64, device="cuda:0")
            for k in keys}


def test_device_requests_equal_direct_calls(env):
    """Requests on device arrays are evaluated in place, chunk by chunk (the species rows of Y
    and hRT keep the request's stride): bit for bit the direct call, for every route and for
    the solver outputs of (h, P, Y)."""
    import torch
    P, mech, net = env
    s = P.Server(mech, net, mem_budget=64 << 20, chunk_cells=1000, streams=3)
    n = 4321                                    # five chunks, the last one ragged
    ins = to_dev(req(n, 21, res=20))
    torch.cuda.synchronize()
    for route, prec in ((P.ROUTE_PR_FP64, P.FP64), (P.ROUTE_PR_MIXED, P.MIXED)):
        o, sd = dev_outputs(n, KEYS10), torch.full((n,), 255, dtype=torch.uint8, device="cuda:0")
        s.wait(s.submit(P.PTY, route, n, ins, o, sd))
        od, sd2 = dev_outputs(n, KEYS10), torch.empty(n, dtype=torch.uint8, device="cuda:0")
        P.pr(mech, P.PTY, prec, ins, od, n, status=sd2)
        torch.cuda.synchronize()
        for k in KEYS10:
            assert torch.equal(o[k].view(torch.int64), od[k].view(torch.int64)), (route, k)
        assert torch.equal(sd, sd2)
    # (h, P, Y) with psi, alpha, hRT and iters
    h = torch.empty(n, dtype=torch.float64, device="cuda:0")
    P.pr(mech, P.PTY, P.FP64, ins, {"h": h}, n)
    hin = {"h": h, "P": ins["P"], "Y": ins["Y"], "T_guess": ins["T"] * 1.004}
    keys = KEYS10 + ("psi", "alpha", "hRT")
    torch.cuda.synchronize()
    o = dev_outputs(n, keys)
    o["iters"] = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    s.wait(s.submit(P.HPY, P.ROUTE_PR_FP64, n, hin, o))
    od = dev_outputs(n, keys)
    od["iters"] = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    P.pr(mech, P.HPY, P.FP64, hin, od, n)
    torch.cuda.synchronize()
    for k in keys + ("iters",):
        assert torch.equal(o[k], od[k]) if k == "iters" else torch.equal(o[k].view(torch.int64), od[k].view(torch.int64)), k
    # the surrogate with its fallback (cells outside the box planted)
    Tb = ins["T"].clone()
    Tb[::7] = 3400.0
    din = {"P": ins["P"], "T": Tb, "Y": ins["Y"]}
    torch.cuda.synchronize()
    o, sd = dev_outputs(n, KEYS6), torch.full((n,), 255, dtype=torch.uint8, device="cuda:0")
    s.wait(s.submit(P.PTY, P.ROUTE_DNN, n, din, o, sd))
    od, sd2 = dev_outputs(n, KEYS6), torch.empty(n, dtype=torch.uint8, device="cuda:0")
    net(din, od, n, fallback=mech, status=sd2)
    torch.cuda.synchronize()
    assert int(((sd2 & 128) != 0).sum()) >= n // 7
    for k in KEYS6:
        assert torch.equal(o[k].view(torch.int64), od[k].view(torch.int64)), k
    assert torch.equal(sd, sd2)
    s.close()


def test_device_alone_equals_in_the_mix(env):
    import torch
    P, mech, net = env
    s = P.Server(mech, net, mem_budget=64 << 20, chunk_cells=2048, streams=4)
    base = to_dev(req(5000, 7, res=20))
    torch.cuda.synchronize()
    cases = [(P.ROUTE_PR_MIXED, KEYS10), (P.ROUTE_DNN, KEYS6), (P.ROUTE_PR_FP64, KEYS10)]

    def submit(route, keys, ins):
        n = ins["Y"].shape[1]
        o, st = dev_outputs(n, keys), torch.zeros(n, dtype=torch.uint8, device="cuda:0")
        return s.submit(P.PTY, route, n, ins, o, st), (o, st)

    alone = []
    for route, keys in cases:
        t, r = submit(route, keys, base)
        s.wait(t)
        alone.append(r)
    rng = np.random.default_rng(9)
    pending, again = [], []
    for j in range(30):
        n = int(rng.integers(1, 5000))
        ins = to_dev(req(n, 200 + j, res=18))
        torch.cuda.synchronize()
        pending.append(submit([P.ROUTE_PR_MIXED, P.ROUTE_DNN, P.ROUTE_PR_FP64][j % 3], KEYS6, ins)[0])
        if j in (4, 17):
            for route, keys in cases:
                t, r = submit(route, keys, base)
                pending.append(t)
                again.append(r)
    for t in pending:
        s.wait(t)
    assert len(again) == 6
    for j, (o2, st2) in enumerate(again):
        o1, st1 = alone[j % 3]
        for k in o1:
            assert torch.equal(o1[k].view(torch.int64), o2[k].view(torch.int64)), (j, k)
        assert torch.equal(st1, st2)
    assert s.stats()["failed"] == 0
    s.close()


def test_dnn_route_refuses_outputs_it_does_not_produce(env):
    """The surrogate predicts rho, h, cp, c, mu and lambda only: a request for T, P, Z or e on
    that route is refused (host and device requests), instead of returning stale memory."""
    P, mech, net = env
    s = P.Server(mech, net, mem_budget=64 << 20, chunk_cells=1024, streams=2)
    ins = req(500, 31, res=12)
    for extra in ("T", "P", "Z", "e"):
        with pytest.raises(P.PropsError, match="EINVAL"):
            s.submit(P.PTY, P.ROUTE_DNN, 500, ins, outputs(500, KEYS6 + (extra,)))
        with pytest.raises(P.PropsError, match="EINVAL"):
            s.submit(P.PTY, P.ROUTE_DNN, 500, to_dev(ins), dev_outputs(500, KEYS6 + (extra,)))
    with pytest.raises(P.PropsError, match="EINVAL"):       # solver outputs need device requests
        s.submit(P.HPY, P.ROUTE_PR_FP64, 500, ins, outputs(500, ("psi",)))
    assert s.stats()["submitted"] == 0
    s.close()
