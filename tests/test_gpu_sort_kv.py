"""GPU parity of the key-value tile sort: keys and values bit-exact against
the oracle's stable sort for every pairs-per-lane setting, tie-heavy and
full-range keys, ragged sizes, in place on the keys, and the workload
size of the key-only tile sort (2^28 pairs)."""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10034_amd import cox

    cox.lib()
    return torch, cox


def up(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pairs(n, kmax, seed):
    g = np.random.default_rng(seed)
    keys = g.integers(0, kmax, n, dtype=np.uint64).astype(np.uint32)
    vals = g.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    return keys, vals


@pytest.mark.parametrize("k", [1, 2, 4, 8])
@pytest.mark.parametrize("n,kmax", [(1, 3), (31, 4), (32, 2), (8191, 16), (256 * 1024 * 4 + 77, 1 << 32),
                                    (3 * 1024 * 1024 + 5, 8)])
def test_tile_sort_kv_matches_oracle(dev, oracle_mod, k, n, kmax):
    torch, cox = dev
    keys, vals = _pairs(n, kmax, n + k)
    print("kv sort", k, n, kmax, flush=True)
    ok, ov = cox.tile_sort_kv(up(torch, keys.view(np.int32)), up(torch, vals.view(np.int32)), cfg=(k, 0))
    wk, wv = oracle_mod.tile_sort_kv_u32(keys, vals)
    assert np.array_equal(ok.cpu().numpy().view(np.uint32), wk)
    assert np.array_equal(ov.cpu().numpy().view(np.uint32), wv)


def test_tile_sort_kv_in_place_keys_and_float_values(dev, oracle_mod):
    torch, cox = dev
    n = 100003
    keys, vals = _pairs(n, 5, 1)
    fv = vals.view(np.float32)
    kd = up(torch, keys.view(np.int32))
    ok, ov = cox.tile_sort_kv(kd, up(torch, fv), out_keys=kd)
    wk, wv = oracle_mod.tile_sort_kv_u32(keys, vals)
    assert np.array_equal(kd.cpu().numpy().view(np.uint32), wk)
    assert np.array_equal(ov.cpu().numpy().view(np.uint32), wv)


def test_tile_sort_kv_rejects_aliased_values(dev):
    torch, cox = dev
    k = torch.zeros(64, dtype=torch.int32, device="cuda")
    v = torch.zeros(64, dtype=torch.int32, device="cuda")
    with pytest.raises(cox.CoxError) as e:
        cox.tile_sort_kv(k, v, out_vals=v)
    assert e.value.code == 1
    with pytest.raises(cox.CoxError) as e:
        cox.tile_sort_kv(k, v, cfg=(16, 0))
    assert e.value.code == 6


def test_tile_sort_kv_full_size(dev, oracle_mod):
    torch, cox = dev
    n = 1 << 28
    print("generating 2^28 pairs", flush=True)
    _, keys, _ = inputs.primitive_inputs(n)
    vals = np.arange(n, dtype=np.uint32)
    print("kv sort 2^28", flush=True)
    ok, ov = cox.tile_sort_kv(up(torch, keys.view(np.int32)), up(torch, vals.view(np.int32)))
    wk, wv = oracle_mod.tile_sort_kv_u32(keys, vals)
    assert np.array_equal(ok.cpu().numpy().view(np.uint32), wk)
    assert np.array_equal(ov.cpu().numpy().view(np.uint32), wv)
