"""GPU parity of the tile sort over groups wider than a warp: 64 keys over a
full wave (one key per lane) or 16 lanes (four keys per lane), and groups
spanning several waves (exchanges through shared memory), bit-exact
against the oracle's per-group sort for ragged sizes, in place, and at
2^28 keys; unsupported shapes are rejected."""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs

pytestmark = pytest.mark.gpu

COMBOS = [(1, 64), (1, 128), (1, 256), (4, 64), (4, 128), (4, 256), (4, 512), (4, 1024)]


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10034_amd import cox

    cox.lib()
    return torch, cox


def up(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("k,tile", COMBOS)
@pytest.mark.parametrize("n", [1, 63, 1024, 3 * 1024 + 17, (1 << 20) + 5])
def test_group_sort_matches_oracle(dev, oracle_mod, k, tile, n):
    torch, cox = dev
    g = np.random.default_rng(n + tile + k)
    keys = g.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    keys[::5] = keys[n // 2]  # ties
    print("group sort", k, tile, n, flush=True)
    got = cox.tile_sort(up(torch, keys.view(np.int32)), tile=tile, cfg=(k, 0)).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle_mod.group_sort_u32(keys, tile))


@pytest.mark.parametrize("k,tile", [(1, 64), (4, 1024)])
def test_group_sort_in_place_and_extremes(dev, oracle_mod, k, tile):
    torch, cox = dev
    n = 50 * tile + 3
    keys = np.tile(np.array([0xFFFFFFFF, 0, 0x80000000, 0x7FFFFFFF], np.uint32), n // 4 + 1)[:n]
    d = up(torch, keys.view(np.int32))
    cox.tile_sort(d, tile=tile, cfg=(k, 0), out=d)
    assert np.array_equal(d.cpu().numpy().view(np.uint32), oracle_mod.group_sort_u32(keys, tile))


def test_group_sort_rejects_unsupported(dev):
    torch, cox = dev
    d = torch.zeros(4096, dtype=torch.int32, device="cuda")
    for tile, k, code in ((48, 4, 1), (2048, 4, 1), (16, 4, 1), (64, 2, 6), (512, 1, 6), (128, 8, 6)):
        with pytest.raises(cox.CoxError) as e:
            cox.tile_sort(d, tile=tile, cfg=(k, 0))
        assert e.value.code == code, (tile, k)


@pytest.mark.parametrize("k,tile", [(1, 64), (4, 1024)])
def test_group_sort_full_size(dev, oracle_mod, k, tile):
    torch, cox = dev
    n = 1 << 28
    print("generating 2^28 keys", flush=True)
    _, keys, _ = inputs.primitive_inputs(n)
    print("group sort 2^28", k, tile, flush=True)
    got = cox.tile_sort(up(torch, keys.view(np.int32)), tile=tile, cfg=(k, 0)).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle_mod.group_sort_u32(keys, tile))
