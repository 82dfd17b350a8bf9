"""GPU tests of the U-Net's non-convolution kernels, each against a float64
CPU computation of its definition (include/sil_unet.h) on the same inputs,
element by element: |gpu - ref| <= bound, where the bound is the kernel's own
rounding (bf16 outputs: half an ulp, 2^-9 relative, doubled for margin) plus
the float32 arithmetic error of the terms it sums (u = 2^-24 per operation
and term, against the sum of the terms' magnitudes).  Integer and selection
results (max pooling and its indices, argmax, the chip input's conversion,
bf16 rounding) are compared bit for bit."""
import ctypes
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24  # float32 unit roundoff
BF = 2.0 ** -8    # twice bf16's half-ulp


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


def _check(got, ref, bound, what):
    got = got.detach().double().cpu()
    ref = ref.double().cpu()
    bound = torch.as_tensor(bound, dtype=torch.float64).cpu()
    err = (got - ref).abs()
    bad = err > bound
    if bad.any():
        i = tuple(int(v) for v in bad.nonzero()[0])
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.numel()} elements out of bound; "
                             f"first {i}: gpu {got[i].item():.7g} ref {ref[i].item():.7g} "
                             f"bound {bound.expand_as(err)[i].item():.3g}")


def _bf(shape, g, scale=1.0):
    return (torch.randn(shape, generator=g) * scale).to(torch.bfloat16)


@pytest.mark.parametrize("P,C", [(512, 8), (4096, 32), (1000, 256)])
def test_bn_relu(un, P, C):
    _say(f"case bn_relu P={P} C={C}")
    g = torch.Generator().manual_seed(P + C)
    z = _bf((P, C), g, 2.0) + torch.linspace(-1, 1, C).to(torch.bfloat16)
    zd = z.double()
    stats = torch.stack([zd.sum(0), (zd * zd).sum(0)]).float()
    gamma = torch.rand(C, generator=g) + 0.5
    beta = torch.randn(C, generator=g) * 0.5
    out = torch.empty((P, C), dtype=torch.bfloat16, device="cuda")
    mr = torch.empty((2, C), device="cuda")
    zc, sc, gc, bc = z.cuda(), stats.cuda(), gamma.cuda(), beta.cuda()
    un._call("sil_unet_bn_relu", un._p(zc), un._p(sc), un._p(gc), un._p(bc),
             ctypes.c_float(1e-5), P, un._p(out), un._p(mr), P, C, un._s())
    torch.cuda.synchronize()
    s = stats.double()
    mean = s[0] / P
    var = (s[1] / P - mean * mean).clamp(min=0)
    rstd = 1.0 / torch.sqrt(var + float(np.float32(1e-5)))
    _check(mr[0], mean, 2 * U32 * mean.abs() + 1e-30, "bn mean")
    _check(mr[1], rstd, 4 * U32 * rstd, "bn rstd")
    m, r = mr[0].double().cpu(), mr[1].double().cpu()
    t = (zd - m) * r * gamma.double()
    y = t + beta.double()
    ref = y.clamp(min=0)
    _check(out, ref, BF * ref + 8 * U32 * (t.abs() + beta.double().abs()), "bn_relu out")


@pytest.mark.parametrize("P,C,scratch", [(512, 8, True), (2048, 64, True), (1000, 256, True),
                                         (3000, 32, False), (1000, 256, False)])
def test_bn_relu_backward(un, P, C, scratch):
    """With scratch the sums are added to dgamma/dbeta; without it they are
    formed in dgamma/dbeta directly (zero on entry)."""
    _say(f"case bn_relu_bwd P={P} C={C} scratch={scratch}")
    g = torch.Generator().manual_seed(7 * P + C)
    z = _bf((P, C), g, 2.0)
    dout = _bf((P, C), g)
    mean = (torch.randn(C, generator=g) * 0.3).float()
    rstd = (torch.rand(C, generator=g) + 0.5).float()
    gamma = torch.rand(C, generator=g) + 0.5
    beta = torch.randn(C, generator=g) * 0.5
    mr = torch.stack([mean, rstd])
    dz = torch.empty((P, C), dtype=torch.bfloat16, device="cuda")
    dgamma = torch.zeros(C, device="cuda")
    dbeta = torch.zeros(C, device="cuda")
    red = torch.empty((2, C), device="cuda") if scratch else None
    zc, dc, mrc, gc, bc = z.cuda(), dout.cuda(), mr.cuda(), gamma.cuda(), beta.cuda()
    un._call("sil_unet_bn_relu_bwd", un._p(dc), un._p(zc), un._p(mrc), un._p(gc), un._p(bc),
             un._p(dz), un._p(dgamma), un._p(dbeta), un._p(red), P, C, un._s())
    torch.cuda.synchronize()
    zh = (z.double() - mean.double()) * rstd.double()
    y = zh * gamma.double() + beta.double()
    # elements whose pre-activation lies within float32 error of 0 may take
    # either side of the ReLU: they widen the sums' bounds by their own terms
    # and their own dz is not checked
    amb = y.abs() <= 8 * U32 * ((zh * gamma.double()).abs() + beta.double().abs())
    zero = torch.zeros(()).double()
    d = torch.where(y > 0, dout.double(), zero)
    da = torch.where(amb, dout.double().abs(), zero)
    s1, s2 = d.sum(0), (d * zh).sum(0)
    e1 = P * U32 * d.abs().sum(0) + da.sum(0)
    e2 = P * U32 * (d * zh).abs().sum(0) + (da * zh.abs()).sum(0)
    _check(dbeta, s1, e1 + 1e-30, "dbeta")
    _check(dgamma, s2, e2 + 1e-30, "dgamma")
    k = gamma.double() * rstd.double()
    ref = k * (d - (s1 + zh * s2) / P)
    bound = BF * ref.abs() + k.abs() * (8 * U32 * (d.abs() + (s1.abs() + zh.abs() * s2.abs()) / P)
                                        + (e1 + zh.abs() * e2) / P)
    bound = torch.where(amb, torch.full((), float("inf")).double(), bound)
    _check(dz, ref, bound, "bn_relu_bwd dz")


def test_affine_relu(un):
    _say("case affine_relu")
    g = torch.Generator().manual_seed(11)
    P, C = 3000, 64
    z = _bf((P, C), g, 3.0)
    scale = torch.rand(C, generator=g) + 0.2
    shift = torch.randn(C, generator=g)
    out = torch.empty((P, C), dtype=torch.bfloat16, device="cuda")
    zc, sc, shc = z.cuda(), scale.cuda(), shift.cuda()
    un._call("sil_unet_affine_relu", un._p(zc), un._p(sc), un._p(shc), un._p(out), P, C, un._s())
    torch.cuda.synchronize()
    t = z.double() * scale.double()
    ref = (t + shift.double()).clamp(min=0)
    _check(out, ref, BF * ref + 4 * U32 * (t.abs() + shift.double().abs()), "affine_relu")


def test_maxpool_forward_and_backward_with_ties(un):
    _say("case maxpool with ties")
    g = torch.Generator().manual_seed(12)
    N, H, W, C = 2, 6, 10, 16
    x = torch.randint(0, 4, (N, H, W, C), generator=g).to(torch.bfloat16)  # many ties
    y = torch.empty((N, H // 2, W // 2, C), dtype=torch.bfloat16, device="cuda")
    idx = torch.empty((N, H // 2, W // 2, C), dtype=torch.uint8, device="cuda")
    xc = x.cuda()
    un._call("sil_unet_maxpool", un._p(xc), un._p(y), un._p(idx), N, H, W, C, un._s())
    dy = _bf((N, H // 2, W // 2, C), g)
    dyc = dy.cuda()
    dx = torch.empty((N, H, W, C), dtype=torch.bfloat16, device="cuda")
    un._call("sil_unet_maxpool_bwd", un._p(dyc), un._p(idx), None, un._p(dx), N, H, W, C, None,
             un._s())
    # with the skip connection's gradient added in the same kernel, in place
    dskip = _bf((N, H, W, C), g)
    dsum = dskip.cuda()
    un._call("sil_unet_maxpool_bwd", un._p(dyc), un._p(idx), un._p(dsum), un._p(dsum), N, H, W, C,
             None, un._s())
    torch.cuda.synchronize()
    # window positions in row-major order; the first maximum wins
    win = torch.stack([x[:, 0::2, 0::2], x[:, 0::2, 1::2], x[:, 1::2, 0::2], x[:, 1::2, 1::2]])
    mx = win.max(0).values
    first = (win == mx.unsqueeze(0)).float().argmax(0).to(torch.uint8)
    assert torch.equal(y.cpu(), mx)
    assert torch.equal(idx.cpu(), first)
    ref = torch.zeros((N, H, W, C), dtype=torch.bfloat16)
    for k, (a, b) in enumerate([(0, 0), (0, 1), (1, 0), (1, 1)]):
        ref[:, a::2, b::2] = torch.where(first == k, dy, torch.zeros((), dtype=torch.bfloat16))
    assert torch.equal(dx.cpu(), ref)
    # the fp32 sum of two bf16 values, rounded once to bf16
    assert torch.equal(dsum.cpu(), (ref.float() + dskip.float()).to(torch.bfloat16))


@pytest.mark.parametrize("P,C", [(777, 8), (2048, 32), (300, 256)])
def test_head_forward_and_backward(un, P, C):
    _say(f"case head P={P} C={C}")
    g = torch.Generator().manual_seed(P * 3 + C)
    x = _bf((P, C), g)
    w = torch.randn((3, C), generator=g) * 0.3
    b = torch.randn(3, generator=g)
    dl = torch.randn((P, 3), generator=g) * 1e-3
    xc, wc, bc, dlc = x.cuda(), w.cuda(), b.cuda(), dl.cuda()
    logits = torch.empty((P, 3), device="cuda")
    un._call("sil_unet_head", un._p(xc), un._p(wc), un._p(bc), un._p(logits), P, C, un._s())
    dx = torch.empty((P, C), dtype=torch.bfloat16, device="cuda")
    dw = torch.zeros((3, C), device="cuda")
    db = torch.zeros(3, device="cuda")
    # the gradient arriving at the loss scales dlogits on the device
    dscale = torch.tensor([1.5], device="cuda")
    un._call("sil_unet_head_bwd", un._p(xc), un._p(wc), un._p(dlc), un._p(dscale), un._p(dx),
             un._p(dw), un._p(db), P, C, None, un._s())
    torch.cuda.synchronize()
    xd, wd, dld = x.double(), w.double(), 1.5 * dl.double()
    ref = xd @ wd.T + b.double()
    _check(logits, ref, (C + 1) * U32 * (xd.abs() @ wd.abs().T + b.double().abs()), "head logits")
    rdx = dld @ wd
    _check(dx, rdx, BF * rdx.abs() + 6 * U32 * (dld.abs() @ wd.abs()), "head dx")
    rdw = dld.T @ xd
    _check(dw, rdw, P * U32 * (dld.abs().T @ xd.abs()) + 1e-30, "head dw")
    _check(db, dld.sum(0), P * U32 * dld.abs().sum(0) + 1e-30, "head db")


def test_softmax_xent(un):
    _say("case softmax_xent")
    g = torch.Generator().manual_seed(13)
    P = 5000
    logits = torch.randn((P, 3), generator=g) * 4
    labels = torch.randint(0, 3, (P,), generator=g).to(torch.uint8)
    scale = 1.0 / P
    lc, yc = logits.cuda(), labels.cuda()
    loss = torch.zeros(1, device="cuda")
    dl = torch.empty((P, 3), device="cuda")
    un._call("sil_unet_softmax_xent", un._p(lc), un._p(yc), un._p(loss), un._p(dl),
             ctypes.c_float(scale), P, un._s())
    torch.cuda.synchronize()
    ld = logits.double()
    lse = torch.logsumexp(ld, 1)
    per = lse - ld.gather(1, labels.long().view(-1, 1)).view(-1)
    # expf/logf and the three-term sums: a few units of float32 roundoff per pixel
    # per pixel: expf, logf and the three-term sum (a few float32 roundoffs);
    # across pixels: a tree inside each block and one atomic per block
    # loss is the scaled sum (scale = 1/P: the mean)
    _check(loss[0], scale * per.sum(), scale * (16 * U32 * (lse.abs() + ld.abs().max(1).values).sum()
           + (np.log2(P) + 64) * U32 * per.sum()), "loss")
    sm = torch.softmax(ld, 1)
    ref = (sm - torch.nn.functional.one_hot(labels.long(), 3).double()) * scale
    _check(dl, ref, 16 * U32 * scale * (sm + 1.0), "dlogits")


@pytest.mark.parametrize("P,C", [(5000, 32), (777, 8), (300, 256)])
def test_head_xent_matches_head_then_softmax(un, P, C):
    """The fused head + loss kernel against sil_unet_head followed by
    sil_unet_softmax_xent (both pinned to float64 above): the same arithmetic
    per pixel, so logits and dlogits are bit-identical; the loss is a sum of
    the same per-block partials in another atomic order (float32 roundoff of
    the block count)."""
    _say(f"case head_xent P={P} C={C}")
    g = torch.Generator().manual_seed(P + C)
    x = _bf((P, C), g)
    w = torch.randn((3, C), generator=g) * 0.3
    b = torch.randn(3, generator=g)
    labels = torch.randint(0, 3, (P,), generator=g).to(torch.uint8)
    xc, wc, bc, yc = x.cuda(), w.cuda(), b.cuda(), labels.cuda()
    scale = 1.0 / P
    logits = torch.empty((P, 3), device="cuda")
    loss0 = torch.zeros(1, device="cuda")
    dl0 = torch.empty((P, 3), device="cuda")
    un._call("sil_unet_head", un._p(xc), un._p(wc), un._p(bc), un._p(logits), P, C, un._s())
    un._call("sil_unet_softmax_xent", un._p(logits), un._p(yc), un._p(loss0), un._p(dl0),
             ctypes.c_float(scale), P, un._s())
    for with_logits in (True, False):
        lg = torch.full((P, 3), float("nan"), device="cuda")
        loss = torch.zeros(1, device="cuda")
        dl = torch.empty((P, 3), device="cuda")
        un._call("sil_unet_head_xent", un._p(xc), un._p(wc), un._p(bc), un._p(yc), un._p(loss),
                 un._p(dl), un._p(lg) if with_logits else None, ctypes.c_float(scale), P, C,
                 un._s())
        torch.cuda.synchronize()
        assert torch.equal(dl, dl0)
        if with_logits:
            assert torch.equal(lg, logits)
        else:
            assert torch.isnan(lg).all()  # left unwritten
        nblk = (P + 255) // 256
        assert abs(loss.item() - loss0.item()) <= 2 * nblk * U32 * abs(loss0.item()) + 1e-30
    with pytest.raises(un.sil.SilError):  # labels missing
        un._call("sil_unet_head_xent", un._p(xc), un._p(wc), un._p(bc), None, un._p(loss0),
                 un._p(dl0), None, ctypes.c_float(scale), P, C, un._s())


def test_argmax_first_maximum(un):
    _say("case argmax")
    g = torch.Generator().manual_seed(14)
    P = 4096
    logits = torch.randint(0, 3, (P, 3), generator=g).float()  # ties on purpose
    out = torch.empty(P, dtype=torch.uint8, device="cuda")
    lc = logits.cuda()
    un._call("sil_unet_argmax", un._p(lc), un._p(out), P, un._s())
    torch.cuda.synchronize()
    mx = logits.max(1, keepdim=True).values
    first = (logits == mx).float().argmax(1).to(torch.uint8)
    assert torch.equal(out.cpu(), first)


def test_adam_step(un):
    _say("case adam")
    g = torch.Generator().manual_seed(15)
    n = 10007
    w = torch.randn(n, generator=g)
    grad = torch.randn(n, generator=g) * 1e-2
    m = torch.randn(n, generator=g) * 1e-3
    v = torch.rand(n, generator=g) * 1e-4
    lr, b1, b2, eps, step = 1e-3, 0.9, 0.999, 1e-8, 3
    wc, gc, mc, vc = w.cuda(), grad.cuda(), m.cuda(), v.cuda()
    wbf = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    un._call("sil_unet_adam", un._p(wc), un._p(gc), un._p(mc), un._p(vc), un._p(wbf), n,
             ctypes.c_float(lr), ctypes.c_float(b1), ctypes.c_float(b2), ctypes.c_float(eps), step,
             un._s())
    torch.cuda.synchronize()
    f = lambda a: float(np.float32(a))
    b1f, b2f = f(b1), f(b2)
    c1, c2 = f(1 - f(b1f ** step)), f(1 - f(b2f ** step))
    gd, md, vd = grad.double(), m.double(), v.double()
    mr = b1f * md + (1 - b1f) * gd
    vr = b2f * vd + (1 - b2f) * gd * gd
    upd = f(lr) * (mr / c1) / (torch.sqrt(vr / c2) + f(eps))
    wr = w.double() - upd
    _check(mc, mr, 4 * U32 * (b1f * md.abs() + gd.abs()), "adam m")
    _check(vc, vr, 4 * U32 * (b2f * vd + gd * gd), "adam v")
    _check(wc, wr, 2 * U32 * wr.abs() + 32 * U32 * upd.abs(), "adam w")
    assert torch.equal(wbf.cpu(), wc.cpu().to(torch.bfloat16))  # bf16 copy: round to nearest even


def test_chips_input_conversion(un):
    _say("case chips_input")
    g = torch.Generator().manual_seed(16)
    H, W, pitch, chip = 40, 50, 52, 16
    scene = torch.randint(0, 10001, (3, H, pitch), generator=g).to(torch.int16)
    origins = torch.tensor([[0, 0], [32, 48], [-8, -4], [16, 20], [39, 49]], dtype=torch.int32)
    n = origins.shape[0]
    out = torch.empty((n, chip, chip, 8), dtype=torch.bfloat16, device="cuda")
    sc, oc = scene.cuda(), origins.cuda()
    inv = np.float32(1.0 / 10000.0)
    un._call("sil_unet_chips_input", un._p(sc), H, W, pitch, un._p(oc), n, chip,
             ctypes.c_float(float(inv)), un._p(out), un._s())
    torch.cuda.synchronize()
    ref = torch.zeros((n, chip, chip, 8), dtype=torch.bfloat16)
    s = scene.numpy().view(np.uint16).astype(np.float32)
    for k, (y0, x0) in enumerate(origins.tolist()):
        for h in range(chip):
            for w_ in range(chip):
                y, x = y0 + h, x0 + w_
                if 0 <= y < H and 0 <= x < W:
                    # the float32 product, then round to nearest even in bf16
                    prod = torch.from_numpy(s[:, y, x] * inv)
                    ref[k, h, w_, :3] = prod.to(torch.bfloat16)
    assert torch.equal(out.cpu(), ref)


def test_to_bf16_and_fill(un):
    _say("case to_bf16 and fill")
    g = torch.Generator().manual_seed(17)
    x = torch.randn(4099, generator=g) * 100
    x[:4] = torch.tensor([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 65504.0])  # ties to even, signed zero
    y = torch.empty(4099, dtype=torch.bfloat16, device="cuda")
    xc = x.cuda()
    un._call("sil_unet_to_bf16", un._p(xc), un._p(y), x.numel(), un._s())
    f = torch.empty(1001, device="cuda")
    un._call("sil_unet_fill_f32", un._p(f), f.numel(), ctypes.c_float(-2.5), un._s())
    torch.cuda.synchronize()
    assert torch.equal(y.cpu().view(torch.int16), x.to(torch.bfloat16).view(torch.int16))
    assert (f.cpu() == -2.5).all()


def test_adam_multi_tensor(un):
    """One launch over 50 tensors (two launches of at most 48), sizes around
    the per-block chunk, against the float64 update of each tensor."""
    _say("case adam_multi")
    g = torch.Generator().manual_seed(18)
    sizes = [1, 7, 1023, 1024, 1025, 4096 + 3] + [int(v) for v in
                                                  torch.randint(1, 3000, (44,), generator=g)]
    lr, b1, b2, eps, step = 1e-3, 0.9, 0.999, 1e-8, 5
    host, dev, items = [], [], []
    for n in sizes:
        t = [torch.randn(n, generator=g), torch.randn(n, generator=g) * 1e-2,
             torch.randn(n, generator=g) * 1e-3, torch.rand(n, generator=g) * 1e-4]
        d = [x.cuda() for x in t]
        host.append(t)
        dev.append(d)
        items.append(un._AdamTensor(d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(),
                                    d[3].data_ptr(), n))
    arr = un._array(un._AdamTensor, items)
    un._call("sil_unet_adam_multi", ctypes.cast(arr, ctypes.c_void_p), len(arr),
             ctypes.c_float(lr), ctypes.c_float(b1), ctypes.c_float(b2), ctypes.c_float(eps),
             step, None, un._s())
    torch.cuda.synchronize()
    f = lambda a: float(np.float32(a))
    b1f, b2f = f(b1), f(b2)
    c1, c2 = f(1 - f(b1f ** step)), f(1 - f(b2f ** step))
    for k, ((w, grad, m, v), (wc, _, mc, vc)) in enumerate(zip(host, dev)):
        gd, md, vd = grad.double(), m.double(), v.double()
        mr = b1f * md + (1 - b1f) * gd
        vr = b2f * vd + (1 - b2f) * gd * gd
        upd = f(lr) * (mr / c1) / (torch.sqrt(vr / c2) + f(eps))
        wr = w.double() - upd
        _check(mc, mr, 4 * U32 * (b1f * md.abs() + gd.abs()), f"adam_multi m[{k}]")
        _check(vc, vr, 4 * U32 * (b2f * vd + gd * gd), f"adam_multi v[{k}]")
        _check(wc, wr, 2 * U32 * wr.abs() + 32 * U32 * upd.abs(), f"adam_multi w[{k}]")


def test_prep_weights_layouts(un):
    """bf16 copies (round to nearest even) and the transposed forms, bit for
    bit: wt[ci][r][s][co] = w[co][2-r][2-s][ci] for 3x3 weights and
    wt[ci][q][co] = w[q][co][ci] for 2x2 up-convolution weights."""
    _say("case prep_weights")
    g = torch.Generator().manual_seed(19)
    specs = [("conv3", 16, 8), ("conv3", 32, 64), ("up2", 24, 48), ("conv3", 8, 40),
             ("up2", 8, 8)]
    keep, items, refs = [], [], []
    for kind, cout, cin in specs:
        shape = (cout, 3, 3, cin) if kind == "conv3" else (2, 2, cout, cin)
        w = torch.randn(shape, generator=g) * 3
        wc = w.cuda()
        wb = torch.empty(shape, dtype=torch.bfloat16, device="cuda")
        tshape = (cin, 3, 3, cout) if kind == "conv3" else (cin, 2, 2, cout)
        wt = torch.empty(tshape, dtype=torch.bfloat16, device="cuda")
        keep += [wc, wb, wt]
        items.append(un._WeightPrep(wc.data_ptr(), wb.data_ptr(), wt.data_ptr(),
                                    un.W_CONV3 if kind == "conv3" else un.W_UP2, cout, cin))
        b = w.to(torch.bfloat16)
        if kind == "conv3":
            t = b.flip(1, 2).permute(3, 1, 2, 0).contiguous()
        else:
            t = b.permute(3, 0, 1, 2).contiguous()
        refs.append((wb, b, wt, t))
    arr = un._array(un._WeightPrep, items)
    un._call("sil_unet_prep_weights", ctypes.cast(arr, ctypes.c_void_p), len(arr), un._s())
    torch.cuda.synchronize()
    for k, (wb, b, wt, t) in enumerate(refs):
        assert torch.equal(wb.cpu().view(torch.int16), b.view(torch.int16)), f"wb[{k}]"
        assert torch.equal(wt.cpu().view(torch.int16), t.view(torch.int16)), f"wt[{k}]"


def test_bn_running_statistics_and_fold(un):
    """EMA of the batch statistics (variance recovered from rstd) and the
    inference scale/shift, against float64 on the same float32 inputs."""
    _say("case bn_ema and bn_fold")
    g = torch.Generator().manual_seed(20)
    mom, eps = 0.1, 1e-5
    layers, host, keep = [], [], []
    for C in (8, 32, 256, 64):
        mean = torch.randn(C, generator=g)
        rstd = torch.rand(C, generator=g) * 3 + 0.2
        rm = torch.randn(C, generator=g)
        rv = torch.rand(C, generator=g) + 0.1
        gamma = torch.rand(C, generator=g) + 0.5
        beta = torch.randn(C, generator=g)
        mr = torch.stack([mean, rstd]).cuda()
        rmc, rvc, gc, bc = rm.cuda(), rv.cuda(), gamma.cuda(), beta.cuda()
        sc, sh = torch.empty(C, device="cuda"), torch.empty(C, device="cuda")
        keep += [mr, rmc, rvc, gc, bc, sc, sh]
        layers.append(un._BnLayer(C, mr.data_ptr(), rmc.data_ptr(), rvc.data_ptr(), gc.data_ptr(),
                                  bc.data_ptr(), sc.data_ptr(), sh.data_ptr()))
        host.append((mean, rstd, rm, rv, gamma, beta, rmc, rvc, sc, sh))
    arr = un._array(un._BnLayer, layers)
    un._call("sil_unet_bn_ema", ctypes.cast(arr, ctypes.c_void_p), len(arr), ctypes.c_float(mom),
             ctypes.c_float(eps), un._s())
    un._call("sil_unet_bn_fold", ctypes.cast(arr, ctypes.c_void_p), len(arr), ctypes.c_float(eps),
             un._s())
    torch.cuda.synchronize()
    m32, e32 = float(np.float32(mom)), float(np.float32(eps))
    for k, (mean, rstd, rm, rv, gamma, beta, rmc, rvc, sc, sh) in enumerate(host):
        var = 1.0 / rstd.double() ** 2 - e32
        rm1 = (1 - m32) * rm.double() + m32 * mean.double()
        rv1 = (1 - m32) * rv.double() + m32 * var
        _check(rmc, rm1, 4 * U32 * (rm.double().abs() + mean.double().abs()), f"running_mean[{k}]")
        _check(rvc, rv1, 8 * U32 * (rv.double().abs() + var.abs() + e32), f"running_var[{k}]")
        # the fold reads the updated float32 running statistics
        rmg, rvg = rmc.cpu().double(), rvc.cpu().double()
        scale = gamma.double() / torch.sqrt(rvg + e32)
        shift = beta.double() - rmg * scale
        _check(sc, scale, 8 * U32 * scale.abs(), f"scale[{k}]")
        _check(sh, shift, 8 * U32 * (beta.double().abs() + (rmg * scale).abs()), f"shift[{k}]")


def _bn_layer(g, P, C):
    """A batch-norm layer's saved state: z [P, C] bf16, mr, gamma, beta."""
    z = _bf((P, C), g, 2.0)
    mean = (torch.randn(C, generator=g) * 0.3).float()
    rstd = (torch.rand(C, generator=g) + 0.5).float()
    gamma = torch.rand(C, generator=g) + 0.5
    beta = torch.randn(C, generator=g) * 0.5
    return z, torch.stack([mean, rstd]), gamma, beta


def _bn_sums_ref(dout, z, mr, gamma, beta):
    """float64 sums of the batch-norm backward and their bounds (as in
    test_bn_relu_backward): d = dout where the ReLU passed."""
    zh = (z.double() - mr[0].double()) * mr[1].double()
    y = zh * gamma.double() + beta.double()
    amb = y.abs() <= 8 * U32 * ((zh * gamma.double()).abs() + beta.double().abs())
    zero = torch.zeros(()).double()
    d = torch.where(y > 0, dout.double(), zero)
    da = torch.where(amb, dout.double().abs(), zero)
    P = d.shape[0]
    s1, s2 = d.sum(0), (d * zh).sum(0)
    e1 = P * U32 * d.abs().sum(0) + da.sum(0)
    e2 = P * U32 * (d * zh).abs().sum(0) + (da * zh.abs()).sum(0)
    return s1, s2, e1, e2, zh, d, amb


class _Req:
    """A sil_unet_bn_grad request on device copies of a layer's state."""

    def __init__(self, un, z, mr, gamma, beta):
        C = z.shape[-1]
        self.t = [z.cuda(), mr.cuda(), gamma.cuda(), beta.cuda()]
        self.s_d = torch.zeros(C, device="cuda")
        self.s_x = torch.zeros(C, device="cuda")
        self.req = un._BnGrad(*(t.data_ptr() for t in self.t), self.s_d.data_ptr(),
                              self.s_x.data_ptr(), C)
        self.addr = ctypes.addressof(self.req)


def _check_bn_sums(un, what, dout_gpu, layer, req):
    z, mr, gamma, beta = layer
    C = z.shape[-1]
    s1, s2, e1, e2, *_ = _bn_sums_ref(dout_gpu.cpu().reshape(-1, C), z.reshape(-1, C), mr, gamma,
                                      beta)
    _check(req.s_d, s1, e1 + 1e-30, what + " sum_d")
    _check(req.s_x, s2, e2 + 1e-30, what + " sum_dxhat")


@pytest.mark.parametrize("N,H,W,cout,c0", [(2, 16, 40, 32, 32), (1, 9, 13, 32, 64),
                                           (2, 8, 8, 16, 8)])
def test_bn_sums_in_conv_input_gradient(un, N, H, W, cout, c0):
    """The input gradient with the batch-norm sums of the layer it belongs to:
    the same dx bit for bit, and sums of it against float64."""
    _say(f"case conv dgrad + bn sums N={N} H={H} W={W} cout={cout} c0={c0}")
    g = torch.Generator().manual_seed(N * 100 + H + c0)
    dy = _bf((N, H, W, cout), g)
    wt = _bf((c0, 3, 3, cout), g, 0.1)
    layer = _bn_layer(g, N * H * W, c0)
    dyc, wtc = dy.cuda(), wt.cuda()
    plain = torch.empty((N, H, W, c0), dtype=torch.bfloat16, device="cuda")
    fused = torch.empty_like(plain)
    un._call("sil_unet_conv3x3_dgrad", un._p(dyc), cout, un._p(wtc), un._p(plain), c0, None, 0,
             N, H, W, None, un._s())
    req = _Req(un, *layer)
    un._call("sil_unet_conv3x3_dgrad", un._p(dyc), cout, un._p(wtc), un._p(fused), c0, None, 0,
             N, H, W, req.addr, un._s())
    torch.cuda.synchronize()
    assert torch.equal(plain.cpu().view(torch.int16), fused.cpu().view(torch.int16))
    _check_bn_sums(un, "conv dgrad", fused, layer, req)


@pytest.mark.parametrize("N,H,W,cin,cout", [(2, 8, 8, 64, 32), (1, 5, 7, 256, 128),
                                            (2, 4, 6, 16, 16)])
def test_bn_sums_in_upconv_input_gradient(un, N, H, W, cin, cout):
    _say(f"case upconv dgrad + bn sums N={N} H={H} W={W} cin={cin} cout={cout}")
    g = torch.Generator().manual_seed(N * 7 + H + cin)
    dy = _bf((N, 2 * H, 2 * W, cout), g)
    wt = _bf((cin, 2, 2, cout), g, 0.2)
    C = cin
    if 256 % (C // 8):
        pytest.skip("channel groups must divide 256")
    layer = _bn_layer(g, N * H * W, cin)
    dyc, wtc = dy.cuda(), wt.cuda()
    plain = torch.empty((N, H, W, cin), dtype=torch.bfloat16, device="cuda")
    fused = torch.empty_like(plain)
    un._call("sil_unet_upconv_dgrad", un._p(dyc), un._p(wtc), un._p(plain), N, H, W, cin, cout,
             None, un._s())
    req = _Req(un, *layer)
    un._call("sil_unet_upconv_dgrad", un._p(dyc), un._p(wtc), un._p(fused), N, H, W, cin, cout,
             req.addr, un._s())
    torch.cuda.synchronize()
    assert torch.equal(plain.cpu().view(torch.int16), fused.cpu().view(torch.int16))
    _check_bn_sums(un, "upconv dgrad", fused, layer, req)


def test_bn_sums_in_pool_and_head_backward(un):
    """Max-pool backward (with the skip gradient added) and head backward
    with the batch-norm sums; then the apply step from given sums against
    float64 (the bound of test_bn_relu_backward)."""
    _say("case maxpool/head backward + bn sums, bn apply")
    g = torch.Generator().manual_seed(31)
    N, H, W, C = 2, 12, 20, 32
    x = _bf((N, H, W, C), g)
    xc = x.cuda()
    y = torch.empty((N, H // 2, W // 2, C), dtype=torch.bfloat16, device="cuda")
    idx = torch.empty((N, H // 2, W // 2, C), dtype=torch.uint8, device="cuda")
    un._call("sil_unet_maxpool", un._p(xc), un._p(y), un._p(idx), N, H, W, C, un._s())
    dyc, dadd = _bf((N, H // 2, W // 2, C), g).cuda(), _bf((N, H, W, C), g).cuda()
    plain = torch.empty((N, H, W, C), dtype=torch.bfloat16, device="cuda")
    fused = torch.empty_like(plain)
    un._call("sil_unet_maxpool_bwd", un._p(dyc), un._p(idx), un._p(dadd), un._p(plain), N, H, W, C,
             None, un._s())
    layer = _bn_layer(g, N * H * W, C)
    req = _Req(un, *layer)
    un._call("sil_unet_maxpool_bwd", un._p(dyc), un._p(idx), un._p(dadd), un._p(fused), N, H, W, C,
             req.addr, un._s())
    torch.cuda.synchronize()
    assert torch.equal(plain.cpu().view(torch.int16), fused.cpu().view(torch.int16))
    _check_bn_sums(un, "maxpool bwd", fused, layer, req)

    P = 3000
    hx = _bf((P, C), g).cuda()
    w = (torch.randn((3, C), generator=g) * 0.3).cuda()
    dl = (torch.randn((P, 3), generator=g) * 1e-3).cuda()
    outs = []
    hlayer = _bn_layer(g, P, C)
    hreq = _Req(un, *hlayer)
    for r in (None, hreq.addr):
        dx = torch.empty((P, C), dtype=torch.bfloat16, device="cuda")
        dw, db = torch.zeros((3, C), device="cuda"), torch.zeros(3, device="cuda")
        un._call("sil_unet_head_bwd", un._p(hx), un._p(w), un._p(dl), None, un._p(dx), un._p(dw),
                 un._p(db), P, C, r, un._s())
        outs.append(dx)
    torch.cuda.synchronize()
    assert torch.equal(outs[0].cpu().view(torch.int16), outs[1].cpu().view(torch.int16))
    _check_bn_sums(un, "head bwd", outs[1], hlayer, hreq)

    # the apply step from the sums formed above
    z, mr, gamma, beta = hlayer
    dz = torch.empty((P, C), dtype=torch.bfloat16, device="cuda")
    zc, mrc, gc, bc = hreq.t
    un._call("sil_unet_bn_relu_bwd_apply", un._p(outs[1]), un._p(zc), un._p(mrc), un._p(gc),
             un._p(bc), un._p(hreq.s_d), un._p(hreq.s_x), un._p(dz), P, C, un._s())
    torch.cuda.synchronize()
    s1, s2, e1, e2, zh, d, amb = _bn_sums_ref(outs[1].cpu(), z, mr, gamma, beta)
    k = gamma.double() * mr[1].double()
    ref = k * (d - (s1 + zh * s2) / P)
    bound = BF * ref.abs() + k.abs() * (8 * U32 * (d.abs() + (s1.abs() + zh.abs() * s2.abs()) / P)
                                        + (e1 + zh.abs() * e2) / P)
    bound = torch.where(amb, torch.full((), float("inf")).double(), bound)
    _check(dz, ref, bound, "bn_relu_bwd_apply dz")
