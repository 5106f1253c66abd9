"""Allocation-free CNN forward (sadmm_cnn_forward_noalloc) against the
allocating entry point (sadmm_cnn_forward) through the C ABI: the same
kernels on the same parameters, so the probability maps must agree bit for
bit.  Two calls in a row, the second on a smaller image, so the second call
runs on a scratch array that still holds the first call's activations."""

import numpy as np
import pytest

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu


def params(Q, C, seed):
    rng = np.random.default_rng(seed)
    p = ocnn.init_params(Q, C, seed=seed)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    return p


@pytest.mark.parametrize("half", [True, False])
def test_noalloc_forward_equals_forward(gpu_lib, half):
    import torch
    Q, C = 8, 32
    p = params(Q, C, seed=5)
    rng = np.random.default_rng(6)
    shapes = [(72, 61), (20, 37)]          # second call smaller; both ragged in 16 x 16 tiles
    xs = [np.abs(rng.standard_normal((Q, H, W))).astype(np.float32) for H, W in shapes]
    # the allocating entry point, one handle per image size
    ref = []
    for (H, W), x in zip(shapes, xs):
        c = gpu_lib.Cnn(Q, C, H, W)
        c.set_params(p)
        c.set_half(half)
        ref.append(c.forward(x))
        c.close()
    # the allocation-free one: a single handle, both sizes
    big = gpu_lib.Cnn(Q, C, *shapes[0])
    big.set_params(p)
    big.set_half(half)
    for (H, W), x, r in zip(shapes, xs, ref):
        xd = torch.from_numpy(x).cuda()
        out = torch.full((H, W), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        big.forward_noalloc(xd, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(f"noalloc half={half} {H}x{W}: max |diff| {np.abs(got - r).max():.3e}")
        assert np.isfinite(got).all()
        assert np.array_equal(got, r)
    big.close()


def test_noalloc_forward_rejects_oversized_image(gpu_lib):
    """More than 512 x 512 pixels is refused on the host, before any launch."""
    import torch
    c = gpu_lib.Cnn(2, 4, 16, 16)
    x = torch.zeros((2, 513, 512), dtype=torch.float32, device="cuda")
    out = torch.zeros((513, 512), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu_lib.SadmmError) as e:
        c.forward_noalloc(x, out)
    assert e.value.code == -2
    c.close()
