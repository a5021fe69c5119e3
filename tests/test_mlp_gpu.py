"""GPU tests of the MLP surrogate: forward and gradient parity with the BF16-emulating
oracle, device-side PR fallback, deterministic checkpoint/resume, and training."""
import os

import numpy as np
import pytest

import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def props():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_04830_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def sp8():
    return synth.load_species(synth.FLAME_SPECIES)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def labelled_states(orc, sp8, n, seed):
    """(P, T, Y) training states with FP64 oracle labels (rho, h, cp, c, mu, lambda)."""
    P, T, Y = synth.training_states(n, seed=seed)
    r = orc.Mech(sp8, synth.synthetic_kij(8)).state_PT(P, T, Y)
    X = np.vstack([P, T, Y])                                     # [10, n]
    L = np.vstack([r["rho"], r["h"], r["cp"], r["c"], r["mu"], r["lambda"]])   # [6, n]
    return X, L


def set_params(net, params):
    for l, (W, b) in enumerate(params):
        net.set_layer(l, W.astype(np.float32), b.astype(np.float32))


def rounded_params(params):
    return [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in params]


def scaled_outputs(o, olo, ohi):
    Yp = np.column_stack([o["rho"], o["h"], o["cp"], o["c"], o["mu"], o["lambda"]])
    S = np.array(Yp, copy=True)
    for j, lg in enumerate(omlp.LOG_OUTPUTS):
        if lg:
            S[:, j] = np.log(S[:, j])
    return (S - olo) / (ohi - olo)


def test_forward_matches_bf16_oracle(props, orc, sp8):
    import torch
    X, L = labelled_states(orc, sp8, 8192, seed=31)
    ilo, ihi, olo, ohi = omlp.fit_scalers(X.T, L.T)
    params = rounded_params(omlp.init_params(np.random.default_rng(5)))
    net = props.Network(seed=1)
    set_params(net, params)
    net.set_scalers(ilo, ihi, olo, ohi)
    n = X.shape[1]
    outs = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in ("rho", "h", "cp", "c", "mu", "lambda")}
    st = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    net({"P": dev(X[0]), "T": dev(X[1]), "Y": dev(X[2:])}, outs, n, status=st)
    torch.cuda.synchronize()
    o = {k: v.cpu().numpy() for k, v in outs.items()}
    assert int(st.max().item()) == 0
    g = scaled_outputs(o, olo, ohi)
    xs = omlp.scale_inputs(X.T, ilo, ihi)
    y16, _ = omlp.forward_bf16(params, xs)
    y64, _ = omlp.forward(params, xs)
    d16 = np.abs(g - y16)
    d64 = np.abs(g - y64)
    print(f"\n[mlp fwd] vs bf16 oracle: max {d16.max():.3e} rms {np.sqrt((d16**2).mean()):.3e}; "
          f"vs fp64 oracle: max {d64.max():.3e}")
    assert d16.max() < 1e-2 and np.sqrt((d16 ** 2).mean()) < 1e-3
    assert d64.max() < 5e-2


@pytest.mark.parametrize("mask", [0x35, 0x3F, 0x00])
def test_gradient_matches_bf16_oracle(props, orc, sp8, mask):
    """The L1 gradient on the scaled targets, for the default log outputs (rho, cp, mu,
    lambda) and for networks that log-transform all or none of their outputs."""
    X, L = labelled_states(orc, sp8, 4096, seed=32)
    if mask == 0x3F:
        L = np.abs(L) + 1.0                       # every target positive
    flags = omlp.log_flags(mask)
    ilo, ihi, olo, ohi = omlp.fit_scalers(X.T, L.T, flags)
    params = rounded_params(omlp.init_params(np.random.default_rng(6)))
    net = props.Network(seed=2)
    net.set_log_outputs(mask)
    set_params(net, params)
    net.set_scalers(ilo, ihi, olo, ohi)
    n = X.shape[1]
    Xd, Ld = dev(X.astype(np.float32)), dev(L.astype(np.float32))
    loss, g = net.grad(Xd, Ld, n)
    xs = omlp.scale_inputs(X.astype(np.float32).astype(np.float64).T, ilo, ihi)
    t = omlp.transform_outputs(L.astype(np.float32).astype(np.float64).T, olo, ohi, flags)
    y, cache = omlp.forward_bf16(params, xs)
    grads = omlp.backward_bf16(params, cache, y, t)
    y64, c64 = omlp.forward(params, xs)
    g64 = omlp.backward(params, c64, y64, t)
    assert loss == pytest.approx(omlp.l1_loss(y, t), rel=1e-3)
    off = 0
    for l, ((dW, db), (dW64, _)) in enumerate(zip(grads, g64)):
        o, i = dW.shape
        gw = g[off:off + o * i].reshape(o, i)
        off += o * i
        gb = g[off:off + o]
        off += o
        rel = np.linalg.norm(gw - dW) / np.linalg.norm(dW)
        cos = float((gw * dW).sum() / (np.linalg.norm(gw) * np.linalg.norm(dW)))
        rel64 = np.linalg.norm(gw - dW64) / np.linalg.norm(dW64)
        relb = np.linalg.norm(gb - db) / max(np.linalg.norm(db), 1e-30)
        print(f"[mlp grad mask {mask:#x}] layer {l}: |dW-dW_bf16|/|dW| {rel:.2e} cos {cos:.6f} vs fp64 {rel64:.2e} db {relb:.2e}")
        assert rel < 2e-2 and cos > 0.999 and relb < 2e-2
    assert off == g.size


def test_training_fits_the_box_of_the_log_targets(props):
    """train_dnn fits the output box on the transformed targets: with every output flagged,
    the box is [log min, log max] of the (float) targets."""
    rng = np.random.default_rng(44)
    n = 2 * 4096 + 77
    X = rng.uniform(0, 1, (10, n)).astype(np.float32)
    Yl = np.exp(rng.normal(-12.0, 2.0, (6, n))).astype(np.float32)
    net = props.Network(seed=4)
    net.set_log_outputs(0x3F)
    net.train(dev(X), dev(Yl), n, epochs=1, batch=4096, lr=1e-3, lr_min=1e-4, seed=3)
    ilo, ihi, olo, ohi = net.get_scalers()
    T = np.log(Yl.astype(np.float64))
    assert np.allclose(olo, T.min(1), rtol=1e-14, atol=0) and np.allclose(ohi, T.max(1), rtol=1e-14, atol=0)
    assert np.array_equal(ilo, X.astype(np.float64).min(1)) and np.array_equal(ihi, X.astype(np.float64).max(1))


def test_training_resume_is_bitwise(props, tmp_path):
    """2 epochs + save/load + 2 epochs == 4 epochs in one go (weights, bit for bit)."""
    rng = np.random.default_rng(40)
    n = 3 * 4096 + 1000
    X = rng.uniform(0, 1, (10, n)).astype(np.float32)
    X[2:] /= X[2:].sum(0, keepdims=True)
    Yl = np.vstack([np.exp(X[0] + X[1]), X[0] - 2 * X[1], 1 + X[2], X[3] * 3, np.exp(-X[4] - 1), 0.1 + X[5]]).astype(np.float32)
    Xd, Yd = dev(X), dev(Yl)
    a = props.Network(seed=9)
    _, la = a.train(Xd, Yd, n, epochs=4, batch=4096, total_epochs=4, seed=3)
    b = props.Network(seed=9)
    _, lb1 = b.train(Xd, Yd, n, epochs=2, batch=4096, total_epochs=4, seed=3)
    path = os.path.join(str(tmp_path), "ck.bin")
    b.save(path)
    c = props.Network.load(path)
    _, lb2 = c.train(Xd, Yd, n, epochs=2, batch=4096, total_epochs=4, seed=3, fit_scalers=False)
    for l in range(5):
        wa, ba = a.get_layer(l)
        wc, bc = c.get_layer(l)
        assert np.array_equal(wa.view(np.int32), wc.view(np.int32)), l
        assert np.array_equal(ba.view(np.int32), bc.view(np.int32)), l
    assert np.array_equal(np.concatenate([lb1, lb2]), la)
    assert la[-1] < la[0]


def test_dnn_fallback_matches_pr_mixed(props, orc, sp8):
    import torch
    X, L = labelled_states(orc, sp8, 4096, seed=33)
    ilo, ihi, olo, ohi = omlp.fit_scalers(X.T, L.T)
    net = props.Network(seed=3)
    net.set_scalers(ilo, ihi, olo, ohi)
    mech = props.Mechanism(sp8, synth.synthetic_kij(8))
    # field cells: some outside the training box (hot/high pressure), one non-physical
    P, T, Y = synth.flame_field(10, seed=2)
    n = T.size
    P = P.copy()
    T = T.copy()
    Y = Y.copy()
    T[::7] = 3300.0            # above the box
    P[::11] = 2.0e7            # above the box
    Y[:, 5] = 0.0              # sum Y = 0: non-physical
    ins = {"P": dev(P), "T": dev(T), "Y": dev(Y)}
    keys = ("rho", "h", "cp", "c", "mu", "lambda")
    o1 = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in keys}
    s1 = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    net(ins, o1, n, fallback=mech, status=s1)
    o0 = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in keys}
    s0 = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    net(ins, o0, n, status=s0)
    op = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in keys}
    sp = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    props.pr(mech, props.PTY, props.MIXED, ins, op, n, status=sp)
    torch.cuda.synchronize()
    s1, s0, sp = s1.cpu().numpy(), s0.cpu().numpy(), sp.cpu().numpy()
    flagged = (s0 & 64) != 0
    assert flagged.sum() >= n // 11 and not flagged.all()
    assert flagged[5] and (s1[5] & 1) and (s1[5] & 128)
    assert np.array_equal(s1[flagged], (sp[flagged] | 64 | 128))
    assert np.all(s1[~flagged] == 0)
    for k in keys:
        a, b0, p = o1[k].cpu().numpy(), o0[k].cpu().numpy(), op[k].cpu().numpy()
        assert np.array_equal(a[~flagged], b0[~flagged]), k
        both = np.isnan(a[flagged]) & np.isnan(p[flagged])
        assert np.all(both | (a[flagged] == p[flagged])), k


def test_label_generation_audited_by_oracle(props, orc, sp8):
    """Training labels come from the GPU FP64 (P,T,Y) path; a 1 % subset is recomputed
    by the oracle."""
    import torch
    n = 200_000
    P, T, Y = synth.training_states(n, seed=3)
    mech = props.Mechanism(sp8, synth.synthetic_kij(8))
    keys = ("rho", "h", "cp", "c", "mu", "lambda")
    o = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in keys}
    st = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    props.pr(mech, props.PTY, props.FP64, {"P": dev(P), "T": dev(T), "Y": dev(Y)}, o, n, status=st)
    torch.cuda.synchronize()
    idx = np.random.default_rng(0).choice(n, n // 100, replace=False)
    ref = orc.Mech(sp8, synth.synthetic_kij(8)).state_PT(P[idx], T[idx], np.ascontiguousarray(Y[:, idx]))
    for k in keys:
        g = o[k].cpu().numpy()[idx]
        scale = ref["h_scale"] if k == "h" else np.abs(ref[k])
        assert np.max(np.abs(g - ref[k]) / scale) < 1e-10, k
    assert int((st != 0).sum().item()) == 0
