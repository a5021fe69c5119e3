"""The serving scheduler on the CPU: the mock executor stands in for the GPU and evaluates a
fixed function of each cell's inputs, so routing, chunking, admission, fairness, latency
statistics and failure isolation are checked without a device."""
import math
import threading
import time

import numpy as np
import pytest

import paper_2312_04830_amd as P

NS = 8
OUTS = ("T", "P", "Z", "rho", "h", "e", "cp", "c", "mu", "lambda")


def make_request(n, seed, mode=P.PTY):
    rng = np.random.default_rng(seed)
    a = rng.uniform(1e6, 2e7, n)
    b = rng.uniform(100, 3000, n)
    Y = rng.dirichlet(np.ones(NS), n).T.copy()
    if mode == P.PTY:
        ins = {"P": a, "T": b, "Y": Y}
    elif mode == P.RHOEY:
        ins = {"rho": a, "e": b, "Y": Y}
    else:
        ins = {"h": a, "P": b, "Y": Y}
    outs = {k: np.full(n, np.nan) for k in OUTS}
    return ins, outs, np.full(n, 255, dtype=np.uint8)


def expected(ins, mode, route):
    a, b = {P.PTY: ("P", "T"), P.RHOEY: ("rho", "e"), P.HPY: ("h", "P")}[mode]
    a, b = ins[a], ins[b]
    ys = sum((i + 1) * ins["Y"][i] for i in range(NS))
    n = a.size
    return {"T": b, "P": a, "Z": ys, "rho": a + 2 * b, "h": a * b, "e": a - b, "cp": ys * 3,
            "c": np.full(n, float(route)), "mu": np.full(n, float(mode)), "lambda": np.arange(n, dtype=float)}


def server(**kw):
    kw.setdefault("executor", P.EXEC_MOCK)
    kw.setdefault("mem_budget", 64 << 20)
    kw.setdefault("chunk_cells", 1000)
    return P.Server(None, **kw)


def test_every_cell_returns_to_its_place():
    s = server(streams=3)
    reqs = []
    for i, (n, mode, route) in enumerate([(1, P.PTY, 0), (999, P.PTY, 1), (1000, P.RHOEY, 0),
                                          (1001, P.HPY, 1), (5432, P.RHOEY, 1), (37, P.HPY, 0)]):
        ins, outs, st = make_request(n, i, mode)
        reqs.append((s.submit(mode, route, n, ins, outs, st), ins, outs, st, mode, route))
    for t, ins, outs, st, mode, route in reqs:
        r = s.wait(t)
        assert r["rc"] == 0 and r["n"] == ins["Y"].shape[1]
        exp = expected(ins, mode, route)
        for k in OUTS:
            np.testing.assert_array_equal(outs[k], exp[k], err_msg=k)
        assert np.all(st == 0)
    st = s.stats()
    assert st["completed"] == 6 and st["failed"] == 0 and st["cells_done"] == 1 + 999 + 1000 + 1001 + 5432 + 37
    s.close()


def test_null_outputs_are_not_written():
    s = server()
    ins, outs, _ = make_request(500, 1)
    only = {"rho": outs["rho"], "h": outs["h"]}
    s.wait(s.submit(P.PTY, 0, 500, ins, only))
    assert not np.isnan(outs["rho"]).any() and np.isnan(outs["cp"]).all()
    s.close()


def test_admission_is_bounded_by_memory():
    """A budget of exactly two slots: never more than two chunks in flight."""
    probe = server(mem_budget=1 << 30)
    slot = probe.stats()["slot_bytes"]
    probe.close()
    s = server(mem_budget=2 * slot + slot // 2, mock_ns_per_cell=2000.0, streams=4)
    assert s.stats()["slots"] == 2
    tickets = []
    for i in range(6):
        ins, outs, st = make_request(2500, 10 + i)
        tickets.append(s.submit(P.PTY, 1, 2500, ins, outs, st))
    peak = 0
    for _ in range(200):
        st = s.stats()
        peak = max(peak, st["inflight_chunks"])
        if st["completed"] == 6:
            break
        time.sleep(0.002)
    for t in tickets:
        s.wait(t)
    assert 1 <= peak <= 2
    s.close()


def test_budget_below_one_slot_is_refused():
    with pytest.raises(P.PropsError) as e:
        server(mem_budget=1000, chunk_cells=100000)
    assert e.value.code == -4


def test_small_request_is_not_starved_by_a_large_one():
    s = server(mem_budget=1 << 30, max_inflight=2, streams=2, mock_ns_per_cell=200.0)
    big_in, big_out, _ = make_request(100_000, 1)       # 100 chunks, ~20 ms of mock work
    small_in, small_out, _ = make_request(50, 2)
    tb = s.submit(P.PTY, 0, 100_000, big_in, big_out)
    time.sleep(0.002)
    ts = s.submit(P.PTY, 0, 50, small_in, small_out)
    rs = s.wait(ts)
    rb = s.wait(tb)
    assert rs["t_done"] < rb["t_done"]
    assert rs["latency_s"] < 0.5 * rb["latency_s"]
    s.close()


def test_latency_percentiles_are_nearest_rank():
    s = server(mock_ns_per_cell=50.0)
    lat = []
    for i in range(37):
        ins, outs, _ = make_request(200 + 97 * i, 100 + i)
        lat.append(s.wait(s.submit(P.PTY, 0, ins["Y"].shape[1], ins, outs))["latency_s"])
    st = s.stats()
    v = sorted(lat)
    rank = lambda p: v[max(0, math.ceil(p * len(v)) - 1)]  # noqa: E731
    assert st["p50_s"] == pytest.approx(rank(0.5), abs=1e-12)
    assert st["p99_s"] == pytest.approx(rank(0.99), abs=1e-12)
    assert st["max_s"] == pytest.approx(v[-1], abs=1e-12)
    assert st["mean_s"] == pytest.approx(sum(v) / len(v), rel=1e-9)
    s.close()


def test_a_failing_request_does_not_stop_the_server():
    s = server(streams=2)
    bad_in, bad_out, _ = make_request(3000, 1)
    bad_in["P"][1000] = np.nan                  # the second chunk is rejected by the executor
    good = [make_request(1500, 10 + i) for i in range(4)]
    tb = s.submit(P.PTY, 0, 3000, bad_in, bad_out)
    tg = [s.submit(P.PTY, 0, 1500, g[0], g[1], g[2]) for g in good]
    with pytest.raises(P.PropsError) as e:
        s.wait(tb)
    assert e.value.code == -1
    for t, (ins, outs, st) in zip(tg, good):
        s.wait(t)
        np.testing.assert_array_equal(outs["rho"], expected(ins, P.PTY, 0)["rho"])
    ins, outs, _ = make_request(10, 99)
    s.wait(s.submit(P.PTY, 1, 10, ins, outs))
    st = s.stats()
    assert st["failed"] == 1 and st["completed"] == 5
    s.close()


def test_invalid_requests_are_refused():
    s = server()
    ins, outs, _ = make_request(10, 1)
    with pytest.raises(P.PropsError):
        s.submit(P.PTY, 0, 0, ins, outs)
    with pytest.raises(P.PropsError):
        s.submit(P.PTY, P.ROUTE_DNN, 10, ins, outs)          # no network
    with pytest.raises(P.PropsError):
        s.submit(P.RHOEY, 0, 10, ins, outs)                   # rho, e missing
    with pytest.raises(P.PropsError):
        s.submit(P.PTY, 7, 10, ins, outs)
    with pytest.raises(P.PropsError):
        s.wait(12345)
    s.close()


def test_wait_times_out_then_completes():
    s = server(mock_ns_per_cell=5000.0, max_inflight=1, streams=1)
    ins, outs, _ = make_request(20_000, 3)                    # ~0.1 s of mock work
    t = s.submit(P.PTY, 0, 20_000, ins, outs)
    with pytest.raises(P.PropsError) as e:
        s.wait(t, timeout_us=0)
    assert e.value.code == -5
    assert s.wait(t)["rc"] == 0
    s.close()


def test_concurrent_submitters():
    s = server(streams=4)
    results = {}

    def client(k):
        ins, outs, _ = make_request(700 + 13 * k, 1000 + k)
        t = s.submit(P.PTY, k % 2, ins["Y"].shape[1], ins, outs)
        s.wait(t)
        results[k] = np.array_equal(outs["h"], expected(ins, P.PTY, k % 2)["h"])

    th = [threading.Thread(target=client, args=(k,)) for k in range(16)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert len(results) == 16 and all(results.values())
    s.close()


def test_close_drains_work_in_flight():
    s = server(mock_ns_per_cell=100.0, max_inflight=2)
    ins, outs, _ = make_request(30_000, 5)
    s.submit(P.PTY, 0, 30_000, ins, outs)
    s.close()
    np.testing.assert_array_equal(outs["rho"], expected(ins, P.PTY, 0)["rho"])


def test_submit_refuses_short_or_mistyped_host_arrays():
    """The binding checks each host array against the cells the server will touch."""
    s = server(streams=1)
    ins, outs, st = make_request(100, 7)
    bad = dict(ins, Y=ins["Y"][:, :50].copy())
    with pytest.raises(ValueError, match="Y"):
        s.submit(P.PTY, 0, 100, bad, outs, st)
    with pytest.raises(ValueError, match="status"):
        s.submit(P.PTY, 0, 100, ins, outs, st.astype(np.float64))
    with pytest.raises(ValueError, match="rho"):
        s.submit(P.PTY, 0, 100, ins, dict(outs, rho=np.zeros(99)), st)
    r = s.wait(s.submit(P.PTY, 0, 100, ins, outs, st))
    assert r["rc"] == 0
    s.close()
