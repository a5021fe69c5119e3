"""Size limits of the C ABI: a cell count beyond what one launch can address is refused
with PROPS_ETOOBIG before anything is launched (the arrays passed here are tiny and are
never touched).  The largest count each entry point accepts is stated in props.h."""
import pytest

pytestmark = pytest.mark.gpu

ETOOBIG = -4
HUGE_GRID = 0x7FFFFFFF * 256 + 1      # one more cell than 2^31 - 1 blocks of 256 lanes
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
    ins = {"P": tiny, "T": tiny, "rho": tiny, "e": tiny, "h": tiny, "Y": tiny}
    with pytest.raises(props.PropsError) as e:
        props.pr(mech, getattr(props, mode), props.FP64, ins, {"T": tiny}, HUGE_GRID)
    assert e.value.code == ETOOBIG


def test_diffusion_refuses_a_grid_beyond_the_launch_limit(props, mech, tiny):
    with pytest.raises(props.PropsError) as e:
        props.diffusion(mech, props.FP64, tiny, tiny, tiny, tiny, HUGE_GRID)
    assert e.value.code == ETOOBIG


def test_surrogate_refuses_counts_beyond_32_bit_indices(props, mech, tiny):
    net = props.Network(seed=1)
    with pytest.raises(props.PropsError) as e:
        net({"P": tiny, "T": tiny, "Y": tiny}, {"rho": tiny}, HUGE_INT, fallback=mech)
    assert e.value.code == ETOOBIG
    with pytest.raises(props.PropsError) as e:
        net.features(tiny, tiny, HUGE_INT)
    assert e.value.code == ETOOBIG
