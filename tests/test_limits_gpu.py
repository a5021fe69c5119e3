"""Size limits of the C ABI: a cell count beyond what one launch can address is refused
with PROPS_ETOOBIG before anything is launched (the arrays passed here are tiny and are
never touched).  The largest count each entry point accepts is stated in props.h.  The
calls go straight to the C functions: the Python binding would already refuse arrays
shorter than the count."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu

ETOOBIG = -4
# one more cell than the largest launch: a dispatch holds at most 2^32 - 1 work-items, and
# 2^32 - 256 is the largest multiple of the 64- and 256-lane blocks below that
HUGE_GRID_PR = (1 << 32) - 256 + 1
HUGE_INT = 0x7FFFFFFF + 1             # beyond a 32-bit cell index


@pytest.fixture(scope="module")
def props():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_04830_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def tiny():
    import torch
    return torch.zeros(16, dtype=torch.float64, device="cuda:0")


@pytest.fixture(scope="module")
def mech(props):
    import synth
    return props.Mechanism(synth.load_species(synth.FLAME_SPECIES))


@pytest.mark.parametrize("mode", ["PTY", "RHOEY", "HPY"])
def test_pr_refuses_a_grid_beyond_the_launch_limit(props, mech, tiny, mode):
    p = tiny.data_ptr()
    pin = props._lib.PropsIn(P=p, T=p, rho=p, e=p, Y=p, h=p)
    pout = props._lib.PropsOut(T=p)
    rc = props.lib().props_pr(mech.handle, getattr(props, mode), props.FP64, ctypes.byref(pin), ctypes.byref(pout),
                              HUGE_GRID_PR, None, None)
    assert rc == ETOOBIG, props.lib().props_last_error()


def test_diffusion_refuses_a_grid_beyond_the_launch_limit(props, mech, tiny):
    p = tiny.data_ptr()
    rc = props.lib().props_diffusion(mech.handle, props.FP64, p, p, p, p, HUGE_GRID_PR, None, None)
    assert rc == ETOOBIG, props.lib().props_last_error()


def test_surrogate_refuses_counts_beyond_32_bit_indices(props, mech, tiny):
    net = props.Network(seed=1)
    p = tiny.data_ptr()
    pin = props._lib.PropsIn(P=p, T=p, Y=p)
    pout = props._lib.PropsOut(rho=p)
    rc = props.lib().props_dnn(net.handle, mech.handle, ctypes.byref(pin), ctypes.byref(pout), HUGE_INT, None, None)
    assert rc == ETOOBIG, props.lib().props_last_error()
    rc = props.lib().props_dnn_features(net.handle, p, p, HUGE_INT, None)
    assert rc == ETOOBIG, props.lib().props_last_error()


def test_binding_refuses_short_host_or_mistyped_arrays(props, mech, tiny):
    """The binding checks each device array against the element count the call will touch."""
    import torch
    ins = {"P": tiny, "T": tiny, "Y": tiny}
    with pytest.raises(ValueError, match="elements"):
        props.pr(mech, props.PTY, props.FP64, ins, {"rho": tiny}, 4)          # Y needs 8 x 4
    with pytest.raises(ValueError, match="device"):
        props.pr(mech, props.PTY, props.FP64, {"P": tiny.cpu(), "T": tiny, "Y": tiny}, {}, 1)
    with pytest.raises(ValueError, match="float64"):
        props.diffusion(mech, props.FP64, tiny.float(), tiny, tiny, tiny, 1)
    with pytest.raises(ValueError, match="status"):
        props.diffusion(mech, props.FP64, tiny, tiny, tiny, tiny, 2, status=torch.zeros(1, dtype=torch.uint8,
                                                                                     device="cuda:0"))


@pytest.mark.parametrize("nbytes", [0, 15, 16, 4096 * 16 + 5, (1 << 22) + 48 + 9])
def test_stream_copy_reproduces_its_source(props, nbytes):
    """The streaming copy (the bandwidth denominator of the benchmark) reproduces every byte,
    whole vectors, the tail trip and the ragged byte tail, and writes nothing past the end."""
    import torch
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, generator=g).to("cuda:0")
    dst = torch.full((nbytes + 64,), 7, dtype=torch.uint8, device="cuda:0")
    props.stream_copy(src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes].cpu(), src[:nbytes].cpu())
    assert bool((dst[nbytes:] == 7).all())


def test_stream_copy_refuses_misaligned_pointers(props):
    import torch
    buf = torch.zeros(256, dtype=torch.uint8, device="cuda:0")
    rc = props.lib().props_stream_copy(ctypes.c_void_p(buf.data_ptr() + 8), ctypes.c_void_p(buf.data_ptr() + 128),
                                       ctypes.c_size_t(64), None)
    assert rc == -1   # PROPS_EINVAL
