"""GPU tests of the U-Net kernels: each MFMA convolution against a float32
CPU reference of the same operation (bf16-exact inputs, so only summation
order differs), the whole network's loss, logits and gradients against the
float64 oracle (oracle/unet_ref.py) on an 8-16 channel variant at 32x32, and
a few training steps lowering the loss."""
import sys

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet_ref as U
from tests import unet_bf16

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def un():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_13135_amd import unet
    unet._lib()
    return unet


def _bf(shape, g, scale=1.0):
    return (torch.randn(shape, generator=g) * scale).to(torch.bfloat16)


def _rel(a, b):
    a = a.double().cpu()
    b = b.double().cpu()
    return (a - b).norm().item() / max(b.norm().item(), 1e-30)


# Shapes reach every tile family: narrow (32-wide) and wide outputs, ragged
# weight-gradient N tiles (9*cin = 72), N tiles of 96/192/128 with 32-, 64- and
# 128-row M tiles, a 256 x 256 batch whose tiles outnumber the resident blocks
# (each block walks several tiles), and images that are not multiples of the
# LDS kernels' 8 x 32 pixel tiles in either direction.
@pytest.mark.parametrize("N,H,W,c0,c1,cout", [(2, 16, 16, 8, 0, 32), (1, 9, 13, 16, 16, 8),
                                              (2, 32, 32, 32, 0, 64), (1, 8, 8, 64, 64, 128),
                                              (3, 4, 4, 128, 0, 256), (1, 16, 16, 32, 32, 32),
                                              (2, 8, 8, 64, 0, 64), (1, 8, 8, 64, 0, 128),
                                              (1, 8, 8, 32, 0, 128), (4, 256, 256, 32, 0, 32),
                                              (2, 9, 45, 32, 32, 64), (1, 17, 33, 64, 0, 32)])
def test_conv3x3_forward_and_gradients(un, N, H, W, c0, c1, cout):
    _say(f"case conv3x3 {N, H, W, c0, c1, cout}")
    g = torch.Generator().manual_seed(N * 1000 + H * 10 + cout)
    x0 = _bf((N, H, W, c0), g)
    x1 = _bf((N, H, W, c1), g) if c1 else None
    w = _bf((cout, 3, 3, c0 + c1), g, 0.1)
    dy = _bf((N, H, W, cout), g)
    x = x0 if x1 is None else torch.cat([x0, x1], dim=3)
    xr = x.float().permute(0, 3, 1, 2).requires_grad_(True)
    wr = w.float().permute(0, 3, 1, 2).requires_grad_(True)
    yr = F.conv2d(xr, wr, padding=1)
    yr.backward(dy.float().permute(0, 3, 1, 2))
    # device copies held in variables for the whole test (no aliasing of freed blocks)
    x0c, wc, dyc = x0.cuda(), w.cuda(), dy.cuda()
    x1c = x1.cuda() if x1 is not None else None
    y = torch.empty((N, H, W, cout), dtype=torch.bfloat16, device="cuda")
    stats = torch.zeros((2, cout), device="cuda")
    un._call("sil_unet_conv3x3", un._p(x0c), c0, un._p(x1c), c1, un._p(wc), un._p(y),
             un._p(stats), N, H, W, cout, un._s())
    wt = torch.empty((c0 + c1, 3, 3, cout), dtype=torch.bfloat16, device="cuda")
    un._call("sil_unet_flip3x3", un._p(wc), un._p(wt), cout, c0 + c1, un._s())
    dx0 = torch.empty((N, H, W, c0), dtype=torch.bfloat16, device="cuda")
    dx1 = torch.empty((N, H, W, c1), dtype=torch.bfloat16, device="cuda") if c1 else None
    un._call("sil_unet_conv3x3_dgrad", un._p(dyc), cout, un._p(wt), un._p(dx0), c0, un._p(dx1),
             c1, N, H, W, un._s())
    dw = torch.zeros((cout, 3, 3, c0 + c1), device="cuda")
    un._call("sil_unet_conv3x3_wgrad", un._p(dyc), cout, un._p(x0c), c0, un._p(x1c), c1,
             un._p(dw), N, H, W, un._s())
    torch.cuda.synchronize()
    yref = yr.detach().permute(0, 2, 3, 1)
    assert _rel(y, yref) < 5e-3  # output rounded to bf16
    assert _rel(stats[0], yref.sum(dim=(0, 1, 2))) < 1e-4 + 1e-3 * yref.abs().sum().item() / max(
        yref.sum(dim=(0, 1, 2)).norm().item(), 1)
    assert _rel(stats[1], (yref * yref).sum(dim=(0, 1, 2))) < 1e-4
    dxr = xr.grad.permute(0, 2, 3, 1)
    assert _rel(dx0, dxr[..., :c0]) < 5e-3
    if c1:
        assert _rel(dx1, dxr[..., c0:]) < 5e-3
    assert _rel(dw, wr.grad.permute(0, 2, 3, 1)) < 1e-4


@pytest.mark.parametrize("N,H,W,c0,c1,cout", [(2, 16, 16, 8, 0, 32), (1, 9, 13, 16, 16, 8),
                                              (2, 32, 32, 64, 64, 128), (3, 64, 64, 32, 0, 32),
                                              (2, 9, 45, 32, 32, 64)])
def test_conv3x3_affine_relu_inference(un, N, H, W, c0, c1, cout):
    """The fused inference layer against a float32 CPU conv, affine and ReLU."""
    _say(f"case conv3x3 affine relu {N, H, W, c0, c1, cout}")
    g = torch.Generator().manual_seed(N * 7 + H + cout)
    x0 = _bf((N, H, W, c0), g)
    x1 = _bf((N, H, W, c1), g) if c1 else None
    w = _bf((cout, 3, 3, c0 + c1), g, 0.1)
    scale = torch.rand(cout, generator=g) + 0.5
    shift = torch.randn(cout, generator=g) * 0.3
    x = x0 if x1 is None else torch.cat([x0, x1], dim=3)
    ref = F.conv2d(x.float().permute(0, 3, 1, 2), w.float().permute(0, 3, 1, 2), padding=1)
    ref = torch.relu(ref * scale.view(1, -1, 1, 1) + shift.view(1, -1, 1, 1)).permute(0, 2, 3, 1)
    x0c, wc, sc, shc = x0.cuda(), w.cuda(), scale.cuda(), shift.cuda()
    x1c = x1.cuda() if x1 is not None else None
    y = torch.empty((N, H, W, cout), dtype=torch.bfloat16, device="cuda")
    un._call("sil_unet_conv3x3_affine_relu", un._p(x0c), c0, un._p(x1c), c1, un._p(wc),
             un._p(sc), un._p(shc), un._p(y), N, H, W, cout, un._s())
    torch.cuda.synchronize()
    assert _rel(y, ref) < 5e-3


@pytest.mark.parametrize("N,H,W,cin,cout", [(2, 8, 8, 16, 8), (1, 5, 7, 64, 32), (2, 16, 16, 256, 128)])
def test_upconv_forward_and_gradients(un, N, H, W, cin, cout):
    _say(f"case upconv {N, H, W, cin, cout}")
    g = torch.Generator().manual_seed(cin + cout + H)
    x = _bf((N, H, W, cin), g)
    w = _bf((2, 2, cout, cin), g, 0.1)
    b = torch.randn(cout, generator=g)
    dy = _bf((N, 2 * H, 2 * W, cout), g)
    xr = x.float().permute(0, 3, 1, 2).requires_grad_(True)
    wr = w.float().permute(3, 2, 0, 1).contiguous().requires_grad_(True)  # [cin, cout, 2, 2]
    br = b.clone().requires_grad_(True)
    yr = F.conv_transpose2d(xr, wr, br, stride=2)
    yr.backward(dy.float().permute(0, 3, 1, 2))
    y = torch.empty((N, 2 * H, 2 * W, cout), dtype=torch.bfloat16, device="cuda")
    xc, wc, bc, dyc = x.cuda(), w.cuda(), b.cuda(), dy.cuda()
    un._call("sil_unet_upconv", un._p(xc), un._p(wc), un._p(bc), un._p(y), N, H, W, cin, cout,
             un._s())
    wt = torch.empty((cin, 2, 2, cout), dtype=torch.bfloat16, device="cuda")
    un._call("sil_unet_up_t", un._p(wc), un._p(wt), cin, cout, un._s())
    dx = torch.empty_like(xc)
    un._call("sil_unet_upconv_dgrad", un._p(dyc), un._p(wt), un._p(dx), N, H, W, cin, cout,
             un._s())
    dw = torch.zeros((2, 2, cout, cin), device="cuda")
    db = torch.zeros((cout,), device="cuda")
    un._call("sil_unet_upconv_wgrad", un._p(xc), un._p(dyc), un._p(dw), un._p(db), N, H, W, cin,
             cout, un._s())
    torch.cuda.synchronize()
    assert _rel(y, yr.detach().permute(0, 2, 3, 1)) < 5e-3
    assert _rel(dx, xr.grad.permute(0, 2, 3, 1)) < 5e-3
    assert _rel(dw, wr.grad.permute(2, 3, 1, 0)) < 1e-4
    assert _rel(db, br.grad) < 1e-4


def _oracle_params(model, widths):
    P = {}
    for k, v in model.params.items():
        t = v.detach().double().cpu()
        if k == "enc0.conv0.w":
            t = t[..., :3]
        elif k.endswith(".up.w"):
            t = t.permute(0, 1, 3, 2)  # [2,2,cout,cin] -> [2,2,cin,cout]
        P[k] = t.contiguous()
    return P


def test_unet_matches_float64_oracle(un):
    widths = (8, 8, 16, 16)
    torch.manual_seed(0)
    model = un.UNet(widths, seed=5)
    g = torch.Generator().manual_seed(6)
    with torch.no_grad():  # non-trivial BN affine and biases
        for k, v in model.params.items():
            if k.endswith((".gamma", ".beta", ".b")):
                v.add_(0.2 * torch.randn(v.shape, generator=g).cuda())
    N, H, W = 2, 32, 32
    x3 = _bf((N, H, W, 3), g)
    x = torch.zeros((N, H, W, 8), dtype=torch.bfloat16)
    x[..., :3] = x3
    labels = torch.randint(0, 3, (N, H, W), generator=g).to(torch.uint8)
    _say("case unet 8-8-16-16 at 32x32 vs float64 oracle")
    loss, logits = model.forward(x.cuda(), labels.cuda())
    loss.backward()
    torch.cuda.synchronize()
    P = _oracle_params(model, widths)
    xo = x3.double().permute(0, 3, 1, 2).contiguous()
    lo, logo, go, _ = U.loss_and_grads(P, xo, labels.long(), widths)
    assert abs(loss.item() - lo.item()) < 0.02 * lo.item()
    assert _rel(logits.permute(0, 3, 1, 2), logo) < 0.05
    # bf16 storage alone (float64 arithmetic, bf16 rounding at the GPU's storage
    # points) moves the gradients by `emul`; the GPU may not do worse than about
    # twice that, layers next to the loss must be tight, and the gradient as a
    # whole must point the same way
    ge = unet_bf16.grads(P, xo, labels, widths)
    flat_g, flat_o = [], []
    bad = {}
    for k, v in model.params.items():
        gg = v.grad.detach().cpu().double()
        if k == "enc0.conv0.w":
            gg = gg[..., :3]
        elif k.endswith(".up.w"):
            gg = gg.permute(0, 1, 3, 2)
        err, emul = _rel(gg, go[k]), _rel(ge[k], go[k])
        if err > max(0.05, 2.0 * emul):
            bad[k] = (round(err, 4), round(emul, 4))
        flat_g.append(gg.reshape(-1))
        flat_o.append(go[k].reshape(-1))
    assert not bad, bad
    for k in ("head.w", "head.b", "dec0.conv1.gamma", "dec0.conv1.beta"):
        gg = model.params[k].grad.detach().cpu().double()
        assert _rel(gg, go[k]) < 0.02, k
    cos = F.cosine_similarity(torch.cat(flat_g), torch.cat(flat_o), dim=0).item()
    assert cos > 0.9, cos


def test_training_steps_reduce_loss(un):
    widths = (8, 16, 16, 32)
    model = un.UNet(widths, seed=1)
    opt = un.Adam(model.params, lr=3e-3)
    g = torch.Generator().manual_seed(2)
    N, H, W = 4, 64, 64
    x = torch.zeros((N, H, W, 8), dtype=torch.bfloat16)
    base = torch.rand((N, H, W), generator=g)
    labels = (base * 3).clamp(max=2.99).long().to(torch.uint8)
    x[..., 0] = (base + 0.05 * torch.randn((N, H, W), generator=g)).to(torch.bfloat16)
    x[..., 1] = x[..., 0]
    x[..., 2] = x[..., 0]
    xc, lc = x.cuda(), labels.cuda()
    losses = []
    for _ in range(30):
        opt.zero_grad()
        loss, _ = model.forward(xc, lc)
        loss.backward()
        opt.step()
        losses.append(loss.item())
    _say(f"losses {losses[0]:.3f} -> {losses[-1]:.3f}")
    assert losses[-1] < 0.5 * losses[0]
