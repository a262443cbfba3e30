"""GPU parity of the integral image: the summed-area table (mod 2^32)
bit-exact against the oracle for single pixels, rows and columns, exact
tiles and tiles plus one, odd widths (the element-wise path), a misaligned
image, and the 8192 x 8192 benchmark image."""
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


# widths that are multiples of 16 take the 16-pixel tile-sum kernel: (3, 2048)
# has fewer rows than its waves, (17, 16) one 16-column group, (8320, 80)
# more than 128 bands (the column pass carries across its batches)
@pytest.mark.parametrize("H,W", [(1, 1), (1, 777), (555, 1), (64, 1024), (65, 1025), (99, 1999), (300, 4099),
                                 (1080, 1920), (2000, 3000), (1999, 3001), (4200, 4200), (3, 2048), (17, 16),
                                 (8320, 80), (4200, 4096)])
def test_integral_image_matches_oracle(dev, oracle_mod, H, W):
    torch, cox = dev
    img = inputs.image_u8(H, W, seed=H + 13 * W)
    if H == 4200:
        img[:] = 255  # the sums wrap past 2^32
    print("integral image", H, W, flush=True)
    got = cox.integral_image(torch.from_numpy(img).cuda()).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle_mod.integral_image_u8(img))


def test_integral_image_misaligned_input(dev, oracle_mod):
    torch, cox = dev
    H, W = 333, 2048
    img = inputs.image_u8(H, W, seed=5)
    buf = torch.zeros(H * W + 1, dtype=torch.uint8, device="cuda")
    buf[1:] = torch.from_numpy(img.reshape(-1)).cuda()
    print("integral image misaligned", flush=True)
    got = cox.integral_image(buf[1:].view(H, W)).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle_mod.integral_image_u8(img))


def test_integral_image_empty(dev):
    torch, cox = dev
    assert cox.integral_image(torch.zeros((0, 7), dtype=torch.uint8, device="cuda")).shape == (0, 7)
    assert cox.integral_image(torch.zeros((7, 0), dtype=torch.uint8, device="cuda")).shape == (7, 0)


def test_integral_image_full_size(dev, oracle_mod):
    torch, cox = dev
    img = inputs.image_u8()
    print("integral image", img.shape, flush=True)
    got = cox.integral_image(torch.from_numpy(img).cuda()).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle_mod.integral_image_u8(img))
