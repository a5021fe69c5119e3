"""GPU tests of the paper-style surrogate inputs: the (h, P, Box-Cox Bilger Z) feature
kernel against the oracle, and inference on raw features (props_dnn_features) against the
BF16-emulating MLP oracle and against props_dnn on the same (P, T, Y) inputs."""
import numpy as np
import pytest

import synth
from oracle import features as of
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

KEYS6 = ("rho", "h", "cp", "c", "mu", "lambda")


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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


@pytest.mark.parametrize("lam", [0.25, 1.0])
def test_features_hpz_match_oracle(props, orc, sp8, lam):
    import torch
    P, T, Y = synth.flame_field(17, seed=2)          # 4913 cells: ragged tail
    n = T.size
    h = orc.Mech(sp8, synth.synthetic_kij(8)).state_PT(P, T, Y, transport=False)["h"]
    X = torch.full((10, n), -7.0, dtype=torch.float64, device="cuda:0")
    props.features_hpz(sp8, 0, 1, lam, dev(h), dev(P), dev(Y), n, X)
    torch.cuda.synchronize()
    g = X.cpu().numpy()
    ref = of.hpz_features(sp8, 0, 1, lam, h, P, Y)
    assert np.array_equal(g[0], ref[0]) and np.array_equal(g[1], ref[1])
    assert np.max(np.abs(g[2] - ref[2])) < 1e-13 * max(1.0, 1.0 / lam)
    assert np.all(g[3:] == 0.0)
    Z = of.bilger_Z(sp8, Y, 0, 1)
    assert Z.min() < 0.01 and Z.max() > 0.99         # the field spans both streams


def test_features_hpz_rejects_bad_arguments(props, sp8):
    import torch
    n = 4
    z = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    Yz = torch.zeros((8, n), dtype=torch.float64, device="cuda:0")
    X = torch.zeros((10, n), dtype=torch.float64, device="cuda:0")
    with pytest.raises(props.PropsError):
        props.features_hpz(sp8, 0, 1, 0.0, z, z, Yz, n, X)      # lambda = 0
    with pytest.raises(props.PropsError):
        props.features_hpz(sp8, 0, 0, 0.5, z, z, Yz, n, X)      # fuel = oxidizer
    with pytest.raises(props.PropsError):
        props.features_hpz(sp8, 0, 9, 0.5, z, z, Yz, n, X)      # index out of range


def test_dnn_features_match_bf16_oracle(props, sp8):
    """A random network on (h, P, BC(Z), 0, ...) features: the seven constant features scale
    to zero on both sides."""
    import torch
    rng = np.random.default_rng(8)
    n = 6000
    X = np.zeros((10, n))
    X[0] = rng.uniform(-6e6, 3e6, n)
    X[1] = rng.uniform(9.9e6, 1.01e7, n)
    X[2] = rng.uniform(-4.0, 0.0, n)
    L = np.abs(rng.normal(1.0, 0.3, (6, n))) + 0.1
    ilo, ihi, olo, ohi = omlp.fit_scalers(X.T, L.T)
    params = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
              for W, b in omlp.init_params(np.random.default_rng(9))]
    net = props.Network(seed=3)
    for l, (W, b) in enumerate(params):
        net.set_layer(l, W.astype(np.float32), b.astype(np.float32))
    net.set_scalers(ilo, ihi, olo, ohi)
    Yd = torch.empty((6, n), dtype=torch.float64, device="cuda:0")
    net.features(dev(X), Yd, n)
    torch.cuda.synchronize()
    g = Yd.cpu().numpy().T
    ys, _ = omlp.forward_bf16(params, omlp.scale_inputs(X.T, ilo, ihi))
    ref = omlp.untransform_outputs(ys, olo, ohi)
    gs = omlp.transform_outputs(g, olo, ohi)
    d = np.abs(gs - ys)
    print(f"\n[dnn features] vs bf16 oracle (scaled): max {d.max():.3e} rms {np.sqrt((d ** 2).mean()):.3e}")
    assert d.max() < 1e-2 and np.sqrt((d ** 2).mean()) < 1e-3
    assert np.all(np.isfinite(g)) and np.all(g[:, [0, 2, 4, 5]] > 0)
    assert ref.shape == g.shape


def test_dnn_features_equal_props_dnn_on_the_same_inputs(props, sp8):
    """Raw (P, T, Y) features through props_dnn_features give props_dnn's outputs bit for bit."""
    import torch
    P, T, Y = synth.flame_field(12, seed=6)
    n = T.size
    net = props.Network(seed=11)
    lo = np.array([P.min(), T.min()] + list(Y.min(1)))
    hi = np.array([P.max(), T.max()] + list(Y.max(1)))
    net.set_scalers(lo, hi, np.array([2.0, -1e7, 7.0, 200.0, -11.5, -3.9]), np.array([7.0, 2e6, 9.5, 1500.0, -8.0, -1.0]))
    outs = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in KEYS6}
    net({"P": dev(P), "T": dev(T), "Y": dev(Y)}, outs, n)
    Yd = torch.empty((6, n), dtype=torch.float64, device="cuda:0")
    net.features(dev(np.vstack([P, T, Y])), Yd, n)
    torch.cuda.synchronize()
    g = Yd.cpu().numpy()
    for j, k in enumerate(KEYS6):
        assert np.array_equal(g[j], outs[k].cpu().numpy()), k


@pytest.mark.parametrize("mask", [0x3F, 0x00, 0x0A])
def test_dnn_features_log_mask_match_bf16_oracle(props, mask):
    """Networks trained on other targets choose which outputs are logarithms: inference
    on raw features applies exp to exactly the flagged outputs."""
    import torch
    rng = np.random.default_rng(20 + mask)
    n = 3000
    X = np.zeros((10, n))
    X[0] = rng.uniform(-6e6, 3e6, n)
    X[1] = rng.uniform(9.9e6, 1.01e7, n)
    X[2] = rng.uniform(-4.0, 0.0, n)
    L = np.exp(rng.normal(-14.0, 1.5, (6, n)))     # positive, spanning decades
    flags = omlp.log_flags(mask)
    ilo, ihi, olo, ohi = omlp.fit_scalers(X.T, L.T, flags)
    params = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
              for W, b in omlp.init_params(np.random.default_rng(mask))]
    net = props.Network(seed=5)
    assert net.get_log_outputs() == 0x35
    net.set_log_outputs(mask)
    assert net.get_log_outputs() == mask
    for l, (W, b) in enumerate(params):
        net.set_layer(l, W.astype(np.float32), b.astype(np.float32))
    net.set_scalers(ilo, ihi, olo, ohi)
    Yd = torch.empty((6, n), dtype=torch.float64, device="cuda:0")
    net.features(dev(X), Yd, n)
    torch.cuda.synchronize()
    g = Yd.cpu().numpy().T
    ys, _ = omlp.forward_bf16(params, omlp.scale_inputs(X.T, ilo, ihi))
    gs = omlp.transform_outputs(g, olo, ohi, flags)
    d = np.abs(gs - ys)
    assert d.max() < 1e-2 and np.sqrt((d ** 2).mean()) < 1e-3
    for j, lg in enumerate(flags):
        if lg:
            assert np.all(g[:, j] > 0)


def test_log_mask_rules_and_checkpoint(props, tmp_path):
    import torch
    net = props.Network(seed=6)
    with pytest.raises(props.PropsError):
        net.set_log_outputs(0x40)                  # beyond output 5
    net.set_log_outputs(0x3F)
    z = torch.ones(4, dtype=torch.float64, device="cuda:0")
    Yz = torch.full((8, 4), 0.125, dtype=torch.float64, device="cuda:0")
    out = {"rho": torch.empty(4, dtype=torch.float64, device="cuda:0")}
    with pytest.raises(props.PropsError):
        net({"P": z, "T": z, "Y": Yz}, out, 4)     # props_dnn needs the (P, T, Y) mask
    path = str(tmp_path / "net.ckpt")
    net.save(path)
    back = props.Network.load(path)
    assert back.get_log_outputs() == 0x3F
