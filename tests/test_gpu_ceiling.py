"""Harness kernels of the measured ceilings (not part of the method): the
streaming copy moves every byte, in one pass and in several, and the VALU
chains leave each lane's eight chains at one."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2202_10647_amd import adkion
    assert torch.cuda.is_available()
    return torch, adkion


@pytest.mark.parametrize("nbytes,reps", [(16, 1), (3 * (1 << 20) + 48, 1), (5 * (1 << 20) + 4080, 3)])
def test_copy_moves_every_byte(env, nbytes, reps):
    torch, ak = env
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    ak.ceiling_copy(dst, src, reps)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_valu_chains(env, kind):
    torch, ak = env
    out = torch.zeros(256 * 40, dtype=torch.float64 if kind == 1 else torch.float32, device="cuda")
    ak.ceiling_valu(kind, 100, out)
    torch.cuda.synchronize()
    assert bool(torch.all(out == 8.0))


def test_ceiling_errors(env):
    torch, ak = env
    a = torch.zeros(40, dtype=torch.uint8, device="cuda")
    with pytest.raises(ak.AdkError) as e:
        ak.ceiling_copy(a, a.clone())  # 40 bytes: not a multiple of 16
    assert e.value.status == ak.ADK_EINVAL
    with pytest.raises(ak.AdkError) as e:
        ak.ceiling_valu(0, 10, torch.zeros(100, dtype=torch.float32, device="cuda"))  # not 256 lanes
    assert e.value.status == ak.ADK_EINVAL
