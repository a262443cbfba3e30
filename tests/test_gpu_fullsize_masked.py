"""Full-size GPU parity of the partial-mask and tile workload: 2^26 int32
elements, the launch configuration the benchmark times, where every block
runs several grid-stride rounds.  Masked shuffles / votes at the three
densities and the tile<T> reductions at T = 4, 8, 16, 32 are compared
element by element with the oracle; so are the dynamic groups' per-element
outputs and per-warp records at D = 512, with the warp-aggregated append
checked as a set plus disjoint per-warp runs."""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs

from test_gpu_dynamic import runs_valid

pytestmark = pytest.mark.gpu

N = 1 << 26


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10034_amd import cox

    cox.lib()
    return torch, cox


@pytest.fixture(scope="module")
def xm():
    print("generating the 2^26 masked-workload input", flush=True)
    return inputs.masked_input(N)


@pytest.fixture(scope="module")
def xg(dev, xm):
    torch, _ = dev
    return torch.from_numpy(xm).cuda()


@pytest.mark.parametrize("D", inputs.MASK_DENSITIES)
def test_masked_full_size(dev, oracle_mod, xm, xg, D):
    torch, cox = dev
    print("masked 2^26 D", D, flush=True)
    out, rec = cox.warp_masked(xg, D)
    oo, orec = oracle_mod.warp_masked(xm, D)
    assert np.array_equal(out.cpu().numpy(), oo)
    assert np.array_equal(rec.cpu().numpy().view(np.uint32), orec)


@pytest.mark.parametrize("T", inputs.TILE_SIZES)
def test_tile_reduce_full_size(dev, oracle_mod, xm, xg, T):
    torch, cox = dev
    print("tile reduce 2^26 T", T, flush=True)
    got = cox.tile_reduce(xg, T).cpu().numpy()
    assert np.array_equal(got, oracle_mod.tile_reduce_i32(xm, T))


def test_dynamic_full_size(dev, oracle_mod, xm, xg):
    torch, cox = dev
    D = 512
    print("dynamic groups 2^26 D", D, flush=True)
    mm, rk, rec, filt, cnt = cox.warp_dynamic(xg, D)
    omm, ork, orec, ofilt, ocnt = oracle_mod.warp_dynamic(xm, D)
    assert np.array_equal(mm.cpu().numpy().view(np.uint32), omm)
    assert np.array_equal(rk.cpu().numpy().view(np.uint32), ork)
    assert np.array_equal(rec.cpu().numpy().view(np.uint32), orec)
    c = int(cnt.cpu()[0])
    assert c == ocnt
    print("checking the append's runs", flush=True)
    runs_valid(filt.cpu().numpy()[:c], xm, D)
