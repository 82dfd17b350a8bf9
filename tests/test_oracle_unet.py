"""Pins of the float64 U-Net oracle (no GPU): finite-difference gradients,
closed forms of the loss and of batch normalisation, and the parameter
count of the 32-64-128-256 network."""
import math

import numpy as np

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


def _np(P):
    return {k: v.numpy() for k, v in P.items()}


def test_forward_wiring_matches_loop_forward():
    # a second forward written with loops from the definitions (tests/unet_loops.py):
    # ReLU placement, pooling, up-convolution, concatenation order and head
    from tests import unet_loops as L
    widths, P, x, _ = _tiny()
    got = U.forward(P, x, widths).numpy()
    ref = L.forward(_np(P), x.numpy(), widths, eps=U.BN_EPS)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_inference_forward_matches_loop_forward():
    from tests import unet_loops as L
    widths, P, x, _ = _tiny()
    g = torch.Generator().manual_seed(9)
    running = {}
    for name, kind, _, cout in U.layer_specs(widths):
        if kind == "conv3":
            running[name] = (0.5 * torch.randn(cout, generator=g, dtype=torch.float64),
                             0.5 + torch.rand(cout, generator=g, dtype=torch.float64))
    got = U.forward(P, x, widths, running=running).numpy()
    ref = L.forward(_np(P), x.numpy(), widths, eps=U.BN_EPS,
                    running={k: (m.numpy(), v.numpy()) for k, (m, v) in running.items()})
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    # running statistics are not batch statistics: the two modes differ
    assert np.abs(got - U.forward(P, x, widths).numpy()).max() > 1e-3


def test_wiring_pin_sees_the_concatenation_order():
    # exchanging the up-sampled and skip halves of a decoder input changes the
    # logits, so the loop forward above would catch a swapped concatenation
    widths, P, x, _ = _tiny()
    Q = dict(P)
    w = P["dec0.conv0.w"]
    c = w.shape[3] // 2
    Q["dec0.conv0.w"] = torch.cat([w[..., c:], w[..., :c]], dim=3)
    assert (U.forward(Q, x, widths) - U.forward(P, x, widths)).abs().max() > 1e-3


def test_loop_helpers_closed_forms():
    from tests import unet_loops as L
    # a 3x3 kernel with a single centre tap copies its channel; pooling takes
    # the window maximum; the up-convolution places x * w in each 2x2 block
    x = np.arange(2 * 3 * 4 * 4, dtype=np.float64).reshape(2, 3, 4, 4)
    w = np.zeros((1, 3, 3, 3))
    w[0, 1, 1, 2] = 1.0
    assert (L.conv3(x, w)[:, 0] == x[:, 2]).all()
    assert (L.maxpool2(x) == x[:, :, 1::2, 1::2]).all()  # increasing along rows and columns
    wu = np.zeros((2, 2, 3, 1))
    wu[1, 0, 1, 0] = 2.0
    y = L.upconv2(x, wu, np.array([0.5]))
    assert (y[:, 0, 1::2, 0::2] == 2.0 * x[:, 1] + 0.5).all()
    assert (y[:, 0, 0::2, :] == 0.5).all()
