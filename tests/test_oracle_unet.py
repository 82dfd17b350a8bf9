"""Pins of the float64 U-Net oracle (no GPU): finite-difference gradients,
closed forms of the loss and of batch normalisation, and the parameter
count of the 32-64-128-256 network."""
import math

import torch
import torch.nn.functional as F

from oracle import unet_ref as U


def _tiny():
    widths = (2, 4)
    P = U.init_params(widths, seed=3)
    g = torch.Generator().manual_seed(4)
    for k in P:  # move BN/bias parameters away from their trivial initial values
        if k.endswith((".gamma", ".beta", ".b")):
            P[k] = P[k] + 0.3 * torch.randn(P[k].shape, generator=g, dtype=torch.float64)
    x = torch.randn(2, 3, 8, 8, generator=g, dtype=torch.float64)
    labels = torch.randint(0, 3, (2, 8, 8), generator=g)
    return widths, P, x, labels


def test_gradients_match_finite_differences():
    widths, P, x, labels = _tiny()
    names = sorted(P)

    def f(*tensors):
        Q = dict(zip(names, tensors[:-1]))
        return U.loss(U.forward(Q, tensors[-1], widths), labels)

    inputs = [P[n].clone().requires_grad_(True) for n in names] + [x.clone().requires_grad_(True)]
    assert torch.autograd.gradcheck(f, inputs, eps=1e-6, atol=1e-5, rtol=1e-4)


def test_loss_of_uniform_logits_is_log3():
    widths, P, x, labels = _tiny()
    P["head.w"] = torch.zeros_like(P["head.w"])
    P["head.b"] = torch.zeros_like(P["head.b"])
    l = U.loss(U.forward(P, x, widths), labels)
    assert abs(l.item() - math.log(3.0)) < 1e-12


def test_batch_norm_normalises_each_channel():
    widths, P, x, _ = _tiny()
    w = P["enc0.conv0.w"].permute(0, 3, 1, 2)
    y = F.conv2d(x, w, padding=1)
    z = F.batch_norm(y, None, None, None, None, training=True, eps=U.BN_EPS)
    m = z.mean(dim=(0, 2, 3))
    v = z.var(dim=(0, 2, 3), unbiased=False)
    assert m.abs().max() < 1e-12
    # var(z) = var(y) / (var(y) + eps)
    vy = y.var(dim=(0, 2, 3), unbiased=False)
    assert torch.allclose(v, vy / (vy + U.BN_EPS), rtol=1e-10)


def test_parameter_count_of_the_32_to_256_network():
    P = U.init_params((32, 64, 128, 256))
    convs = sum(v.numel() for k, v in P.items() if k.endswith(".w"))
    # 3x3 convs: 9*(3*32 + 32*32 + 32*64 + 64*64 + 64*128 + 128*128 + 128*256 + 256*256
    #              + 256*128 + 128*128 + 128*64 + 64*64 + 64*32 + 32*32); up-convs 4*(256*128 +
    #              128*64 + 64*32); head 32*3
    c3 = 9 * (3 * 32 + 32 * 32 + 32 * 64 + 64 * 64 + 64 * 128 + 128 * 128 + 128 * 256 + 256 * 256
              + 256 * 128 + 128 * 128 + 128 * 64 + 64 * 64 + 64 * 32 + 32 * 32)
    up = 4 * (256 * 128 + 128 * 64 + 64 * 32)
    assert convs == c3 + up + 32 * 3
    assert 1.9e6 < convs < 2.0e6


def test_forward_shapes():
    P = U.init_params((8, 16))
    x = torch.randn(1, 3, 32, 32, dtype=torch.float64)
    assert U.forward(P, x, (8, 16)).shape == (1, 3, 32, 32)
