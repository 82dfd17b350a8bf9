"""U-Net trained on the auto-labels (arXiv 2403.13135, section III-C), on the
gfx950 kernels of ``include/sil_unet.h``.

Every layer is a ``torch.autograd.Function`` whose forward and backward call
the library's kernels (BF16 MFMA convolutions with fp32 accumulation, fp32
batch-norm statistics, softmax and loss); torch only holds the tensors and
records the graph.  Activations are bf16 NHWC; master weights are fp32.

Network (widths e.g. 32, 64, 128, 256): per encoder level two 3x3 conv +
batch norm + ReLU and a 2x2 max pool; a bottleneck of two such convolutions;
per decoder level a 2x2 up-convolution (stride 2) halving the channels,
concatenation with the skip map and two 3x3 conv + BN + ReLU; a 1x1 head to
3 classes and softmax cross-entropy.  The 3 input bands are padded to 8
channels with zeros.
"""
import ctypes
import math
from typing import Dict, Sequence

import torch

from . import sil

IN_CH = 8  # input channels after zero padding of the 3 bands
BN_EPS = 1e-5

_bound = False


def _lib():
    global _bound
    L = sil.lib()
    if not _bound:
        vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        sig = {
            "sil_unet_conv3x3": [vp, i32, vp, i32, vp, vp, vp, i32, i32, i32, i32, vp],
            "sil_unet_conv3x3_affine_relu": [vp, i32, vp, i32, vp, vp, vp, vp, i32, i32, i32,
                                             i32, vp],
            "sil_unet_conv3x3_dgrad": [vp, i32, vp, vp, i32, vp, i32, i32, i32, i32, vp, vp],
            "sil_unet_conv3x3_wgrad": [vp, i32, vp, i32, vp, i32, vp, i32, i32, i32, vp],
            "sil_unet_flip3x3": [vp, vp, i32, i32, vp],
            "sil_unet_upconv": [vp, vp, vp, vp, i32, i32, i32, i32, i32, vp],
            "sil_unet_upconv_dgrad": [vp, vp, vp, i32, i32, i32, i32, i32, vp, vp],
            "sil_unet_upconv_wgrad": [vp, vp, vp, vp, i32, i32, i32, i32, i32, vp],
            "sil_unet_up_t": [vp, vp, i32, i32, vp],
            "sil_unet_bn_relu": [vp, vp, vp, vp, f32, i64, vp, vp, i64, i32, vp],
            "sil_unet_bn_relu_bwd": [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, i32, vp],
            "sil_unet_bn_relu_bwd_apply": [vp, vp, vp, vp, vp, vp, vp, vp, i64, i32, vp],
            "sil_unet_affine_relu": [vp, vp, vp, vp, i64, i32, vp],
            "sil_unet_scatter_argmax": [vp, vp, i32, i32, vp, i32, i32, i64, vp],
            "sil_unet_maxpool": [vp, vp, vp, i32, i32, i32, i32, vp],
            "sil_unet_maxpool_bwd": [vp, vp, vp, vp, i32, i32, i32, i32, vp, vp],
            "sil_unet_head": [vp, vp, vp, vp, i64, i32, vp],
            "sil_unet_softmax_xent": [vp, vp, vp, vp, f32, i64, vp],
            "sil_unet_head_xent": [vp, vp, vp, vp, vp, vp, vp, f32, i64, i32, vp],
            "sil_unet_head_bwd": [vp, vp, vp, vp, vp, vp, vp, i64, i32, vp, vp],
            "sil_unet_argmax": [vp, vp, i64, vp],
            "sil_unet_chips_input": [vp, i32, i32, i64, vp, i32, i32, f32, vp, vp],
            "sil_unet_adam": [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp],
            "sil_unet_adam_multi": [vp, i32, f32, f32, f32, f32, i32, vp, vp],
            "sil_unet_counter_add": [vp, i32, vp],
            "sil_unet_prep_weights": [vp, i32, vp],
            "sil_unet_bn_ema": [vp, i32, f32, f32, vp],
            "sil_unet_bn_fold": [vp, i32, f32, vp],
            "sil_unet_to_bf16": [vp, vp, i64, vp],
            "sil_unet_fill_f32": [vp, i64, f32, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _bound = True
    return L


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _call(name, *args):
    rc = getattr(_lib(), name)(*args)
    if rc != sil.OK:
        raise sil.SilError(rc, f"{name}: {sil.strerror(rc)}")


def _bf16(w: torch.Tensor) -> torch.Tensor:
    out = torch.empty(w.shape, dtype=torch.bfloat16, device=w.device)
    _call("sil_unet_to_bf16", _p(w.contiguous()), _p(out), w.numel(), _s())
    return out


class _AdamTensor(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("g", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("n", ctypes.c_int64)]


W_CONV3, W_UP2 = 1, 2


class _WeightPrep(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("wb", ctypes.c_void_p), ("wt", ctypes.c_void_p),
                ("kind", ctypes.c_int32), ("cout", ctypes.c_int32), ("cin", ctypes.c_int32)]


class _BnLayer(ctypes.Structure):
    _fields_ = [("C", ctypes.c_int32), ("mr", ctypes.c_void_p), ("running_mean", ctypes.c_void_p),
                ("running_var", ctypes.c_void_p), ("gamma", ctypes.c_void_p),
                ("beta", ctypes.c_void_p), ("scale", ctypes.c_void_p), ("shift", ctypes.c_void_p)]


class _BnGrad(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("mr", ctypes.c_void_p), ("gamma", ctypes.c_void_p),
                ("beta", ctypes.c_void_p), ("sum_d", ctypes.c_void_p),
                ("sum_dxhat", ctypes.c_void_p), ("C", ctypes.c_int32)]


class _BnSlot:
    """Links a conv + batch-norm + ReLU layer to the one consumer of its
    output.  The layer's forward records its batch-norm input and statistics
    here; the consumer's backward, while it writes the layer's output
    gradient, also forms the layer's batch-norm sums (the beta and gamma
    gradients) in `sums`; the layer's backward then only applies them."""
    __slots__ = ("bn", "sums")

    def __init__(self):
        self.bn = None
        self.sums = None

    def request(self, pool):
        """(address of a sil_unet_bn_grad, the struct to keep alive), or
        (None, None) when the layer recorded nothing."""
        if self.bn is None:
            return None, None
        z, mr, gamma, beta = self.bn
        C = z.shape[-1]
        s_d = _zeros((C,), z.device, pool)
        s_x = _zeros((C,), z.device, pool)
        self.sums = (s_d, s_x)
        req = _BnGrad(z.data_ptr(), mr.data_ptr(), gamma.data_ptr(), beta.data_ptr(),
                      s_d.data_ptr(), s_x.data_ptr(), C)
        return ctypes.addressof(req), req


def _array(ctype, items):
    arr = (ctype * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


class _ZeroPool:
    """Zeroed fp32 scratch for one training step: the batch-norm sums and the
    gradient accumulators of a step are slices of one buffer cleared by a single
    fill at the start of the step, instead of one fill launch per tensor.  A
    step that needs more than the pool holds gets fresh zeroed tensors for the
    rest, and the pool grows to that size at the next step."""

    def __init__(self):
        self.buf = None
        self.used = 0
        self.need = 0
        self.active = False

    def begin_step(self, device):
        self.need = max(self.need, self.used)
        if self.buf is None or self.buf.device != device or self.buf.numel() < self.need:
            self.buf = torch.empty((max(self.need, 1 << 16),), dtype=torch.float32, device=device)
        n = max(self.need, 1)
        _call("sil_unet_fill_f32", _p(self.buf), n, ctypes.c_float(0.0), _s())
        self.used = 0
        self.active = True

    def take(self, shape, device):
        n = 1
        for d in shape:
            n *= int(d)
        start = (self.used + 63) // 64 * 64  # 256-byte aligned slices
        self.used = start + n
        if not self.active or self.buf.device != device or self.used > self.buf.numel() \
                or self.used > max(self.need, 1):
            return None
        return self.buf[start:start + n].view(shape)


def _zeros(shape, device, pool: "_ZeroPool" = None):
    t = pool.take(shape, device) if pool is not None and pool.active else None
    if t is not None:
        return t
    t = torch.empty(shape, dtype=torch.float32, device=device)
    _call("sil_unet_fill_f32", _p(t), t.numel(), ctypes.c_float(0.0), _s())
    return t


class Conv3x3BNReLU(torch.autograd.Function):
    """relu(batchnorm(conv3x3(concat(x0, x1)))) with batch statistics.  wb and
    wt are the weights' bf16 copy and flipped, transposed bf16 form, prepared
    from w for this pass (UNet.prepare_weights)."""

    @staticmethod
    def forward(ctx, x0, x1, w, gamma, beta, mr=None, pool=None, wb=None, wt=None, slot=None,
                in_slot=None):
        """mr (optional [2, cout] fp32) receives the batch (mean, rstd).  slot
        (optional _BnSlot): this layer's link to the one consumer of its
        output; in_slot: the link of the layer that produced x0, when this
        layer is its only consumer."""
        N, H, W, c0 = x0.shape
        c1 = 0 if x1 is None else x1.shape[3]
        cout = w.shape[0]
        if wb is None:
            wb = _bf16(w)
        z = torch.empty((N, H, W, cout), dtype=torch.bfloat16, device=x0.device)
        ctx.pool = pool
        stats = _zeros((2, cout), x0.device, pool)
        _call("sil_unet_conv3x3", _p(x0), c0, _p(x1), c1, _p(wb), _p(z), _p(stats), N, H, W,
              cout, _s())
        out = torch.empty_like(z)
        if mr is None:
            mr = torch.empty((2, cout), dtype=torch.float32, device=x0.device)
        P = N * H * W
        _call("sil_unet_bn_relu", _p(z), _p(stats), _p(gamma), _p(beta), ctypes.c_float(BN_EPS),
              P, _p(out), _p(mr), P, cout, _s())
        ctx.save_for_backward(x0, x1 if x1 is not None else torch.empty(0), wb, z, mr, gamma, beta)
        ctx.wt = wt
        ctx.has_x1 = x1 is not None
        ctx.slot, ctx.in_slot = slot, in_slot
        if slot is not None:
            slot.bn = (z, mr, gamma, beta)
        return out

    @staticmethod
    def backward(ctx, dout):
        x0, x1, wb, z, mr, gamma, beta = ctx.saved_tensors
        x1 = x1 if ctx.has_x1 else None
        dout = dout.contiguous()
        N, H, W, c0 = x0.shape
        c1 = 0 if x1 is None else x1.shape[3]
        cout = wb.shape[0]
        P = N * H * W
        dz = torch.empty_like(z)
        if ctx.slot is not None and ctx.slot.sums is not None:
            # the consumer formed the batch-norm sums while writing dout
            dbeta, dgamma = ctx.slot.sums
            _call("sil_unet_bn_relu_bwd_apply", _p(dout), _p(z), _p(mr), _p(gamma), _p(beta),
                  _p(dbeta), _p(dgamma), _p(dz), P, cout, _s())
        else:
            # fresh zeroed gradients: the batch-norm sums are formed in them directly
            dgamma = _zeros((cout,), z.device, ctx.pool)
            dbeta = _zeros((cout,), z.device, ctx.pool)
            _call("sil_unet_bn_relu_bwd", _p(dout), _p(z), _p(mr), _p(gamma), _p(beta), _p(dz),
                  _p(dgamma), _p(dbeta), None, P, cout, _s())
        dw = _zeros(wb.shape, z.device, ctx.pool)
        _call("sil_unet_conv3x3_wgrad", _p(dz), cout, _p(x0), c0, _p(x1), c1, _p(dw), N, H, W,
              _s())
        dx0 = dx1 = None
        if ctx.needs_input_grad[0] or (x1 is not None and ctx.needs_input_grad[1]):
            wt = ctx.wt
            if wt is None:
                wt = torch.empty((c0 + c1, 3, 3, cout), dtype=torch.bfloat16, device=z.device)
                _call("sil_unet_flip3x3", _p(wb), _p(wt), cout, c0 + c1, _s())
            dx0 = torch.empty_like(x0)
            dx1 = torch.empty_like(x1) if x1 is not None else None
            req, keep = (None, None)
            if ctx.in_slot is not None and x1 is None:
                req, keep = ctx.in_slot.request(ctx.pool)
            _call("sil_unet_conv3x3_dgrad", _p(dz), cout, _p(wt), _p(dx0), c0, _p(dx1), c1, N, H,
                  W, req, _s())
        return dx0, dx1, dw, dgamma, dbeta, None, None, None, None, None, None


class MaxPool2(torch.autograd.Function):
    """2x2 max pooling that also hands its input on unchanged as the skip map:
    returns (pooled, skip).  The gradients of both outputs reach one backward
    call, where the routed pooled gradient and the skip gradient are summed in
    one kernel."""

    @staticmethod
    def forward(ctx, x, in_slot=None, pool=None):
        """in_slot (optional _BnSlot): the link of the layer that produced x;
        its batch-norm sums are formed here in the backward pass."""
        N, H, W, C = x.shape
        y = torch.empty((N, H // 2, W // 2, C), dtype=x.dtype, device=x.device)
        idx = torch.empty((N, H // 2, W // 2, C), dtype=torch.uint8, device=x.device)
        _call("sil_unet_maxpool", _p(x), _p(y), _p(idx), N, H, W, C, _s())
        ctx.save_for_backward(idx)
        ctx.shape = x.shape
        ctx.in_slot, ctx.pool = in_slot, pool
        ctx.set_materialize_grads(False)
        return y, x

    @staticmethod
    def backward(ctx, dy, dskip):
        (idx,) = ctx.saved_tensors
        N, H, W, C = ctx.shape
        if dy is None:
            return dskip, None, None
        dx = torch.empty(ctx.shape, dtype=dy.dtype, device=dy.device)
        dadd = None if dskip is None else dskip.contiguous()
        req, keep = (None, None) if ctx.in_slot is None else ctx.in_slot.request(ctx.pool)
        _call("sil_unet_maxpool_bwd", _p(dy.contiguous()), _p(idx), _p(dadd), _p(dx), N, H, W, C,
              req, _s())
        return dx, None, None


class UpConv2(torch.autograd.Function):
    """2x2 transposed convolution, stride 2, with bias; w: [2, 2, cout, cin].
    wb and wt: the weights' bf16 copy and [cin, 2, 2, cout] bf16 form, prepared
    for this pass (UNet.prepare_weights)."""

    @staticmethod
    def forward(ctx, x, w, b, pool=None, wb=None, wt=None, in_slot=None):
        ctx.pool = pool
        ctx.in_slot = in_slot
        N, H, W, cin = x.shape
        cout = w.shape[2]
        if wb is None:
            wb = _bf16(w)
        y = torch.empty((N, 2 * H, 2 * W, cout), dtype=torch.bfloat16, device=x.device)
        _call("sil_unet_upconv", _p(x), _p(wb), _p(b), _p(y), N, H, W, cin, cout, _s())
        ctx.save_for_backward(x, wb)
        ctx.wt = wt
        return y

    @staticmethod
    def backward(ctx, dy):
        x, wb = ctx.saved_tensors
        dy = dy.contiguous()
        N, H, W, cin = x.shape
        cout = wb.shape[2]
        dw = _zeros(wb.shape, x.device, ctx.pool)
        db = _zeros((cout,), x.device, ctx.pool)
        _call("sil_unet_upconv_wgrad", _p(x), _p(dy), _p(dw), _p(db), N, H, W, cin, cout, _s())
        wt = ctx.wt
        if wt is None:
            wt = torch.empty((cin, 2, 2, cout), dtype=torch.bfloat16, device=x.device)
            _call("sil_unet_up_t", _p(wb), _p(wt), cin, cout, _s())
        dx = torch.empty_like(x)
        req, keep = (None, None) if ctx.in_slot is None else ctx.in_slot.request(ctx.pool)
        _call("sil_unet_upconv_dgrad", _p(dy), _p(wt), _p(dx), N, H, W, cin, cout, req, _s())
        return dx, dw, db, None, None, None, None


class HeadXent(torch.autograd.Function):
    """Mean softmax cross-entropy of the 1x1 head (head and loss in one
    kernel); returns (loss, logits), logits empty unless with_logits."""

    @staticmethod
    def forward(ctx, x, w, b, labels, pool=None, in_slot=None, with_logits=True):
        N, H, W, C = x.shape
        ctx.in_slot = in_slot
        P = N * H * W
        logits = torch.empty((P, 3) if with_logits else (0, 3), dtype=torch.float32,
                             device=x.device)
        ctx.pool = pool
        loss = _zeros((1,), x.device)  # its own tensor: callers may keep it past the step
        dlogits = torch.empty((P, 3), dtype=torch.float32, device=x.device)
        _call("sil_unet_head_xent", _p(x), _p(w), _p(b), _p(labels), _p(loss), _p(dlogits),
              _p(logits) if with_logits else None, ctypes.c_float(1.0 / P), P, C, _s())
        ctx.save_for_backward(x, w, dlogits)
        ctx.mark_non_differentiable(logits)
        ctx.set_materialize_grads(False)
        return loss.view(()), logits.view(N, H, W, 3) if with_logits else logits

    @staticmethod
    def backward(ctx, dloss, _dlogits):
        x, w, dlogits = ctx.saved_tensors
        N, H, W, C = x.shape
        P = N * H * W
        dx = torch.empty_like(x)
        dw = _zeros((3, C), x.device, ctx.pool)
        db = _zeros((3,), x.device, ctx.pool)
        if dloss is None:
            dx.zero_()
            return dx, dw, db, None, None, None, None
        # dlogits carries the 1/P of the mean; the kernel scales it by the
        # incoming gradient on the device (no host synchronisation)
        dl = dloss.contiguous()
        req, keep = (None, None) if ctx.in_slot is None else ctx.in_slot.request(ctx.pool)
        _call("sil_unet_head_bwd", _p(x), _p(w), _p(dlogits), _p(dl), _p(dx), _p(dw), _p(db), P, C,
              req, _s())
        return dx, dw, db, None, None, None, None


def layer_specs(widths: Sequence[int], in_ch: int = IN_CH):
    specs = []
    c = in_ch
    for i, w in enumerate(widths):
        name = f"enc{i}" if i < len(widths) - 1 else "mid"
        specs.append((f"{name}.conv0", "conv3", c, w))
        specs.append((f"{name}.conv1", "conv3", w, w))
        c = w
    for i in reversed(range(len(widths) - 1)):
        w = widths[i]
        specs.append((f"dec{i}.up", "up2", c, w))
        specs.append((f"dec{i}.conv0", "conv3", 2 * w, w))
        specs.append((f"dec{i}.conv1", "conv3", w, w))
        c = w
    specs.append(("head", "conv1", c, 3))
    return specs


class UNet:
    """Parameters (fp32 master copies, GPU) and the forward pass."""

    def __init__(self, widths: Sequence[int], device="cuda", seed: int = 0):
        self.widths = tuple(widths)
        g = torch.Generator().manual_seed(seed)
        P: Dict[str, torch.Tensor] = {}
        for name, kind, cin, cout in layer_specs(widths):
            if kind == "conv3":
                fan = 9 * (3 if name == "enc0.conv0" else cin)
                w = torch.randn(cout, 3, 3, cin, generator=g) * math.sqrt(2.0 / fan)
                if name == "enc0.conv0":
                    w[..., 3:] = 0.0  # padding channels
                P[name + ".w"] = w
                P[name + ".gamma"] = torch.ones(cout)
                P[name + ".beta"] = torch.zeros(cout)
            elif kind == "up2":
                P[name + ".w"] = torch.randn(2, 2, cout, cin, generator=g) * math.sqrt(2.0 / cin)
                P[name + ".b"] = torch.zeros(cout)
            else:
                P[name + ".w"] = torch.randn(cout, cin, generator=g) * math.sqrt(2.0 / cin)
                P[name + ".b"] = torch.zeros(cout)
        self.params = {k: v.to(device).float().requires_grad_(True) for k, v in P.items()}
        self.pool = _ZeroPool()  # this model's per-step zeroed scratch
        # running batch-norm statistics for inference, and the last batch's (mean, rstd)
        self.bn_names = [n for n, kind, _, _ in layer_specs(widths) if kind == "conv3"]
        self.running = {n: (torch.zeros(P[n + ".gamma"].numel(), device=device),
                            torch.ones(P[n + ".gamma"].numel(), device=device))
                        for n in self.bn_names}
        self.batch_mr = {n: torch.empty((2, P[n + ".gamma"].numel()), device=device)
                         for n in self.bn_names}
        self.momentum = 0.1
        # bf16 weights for the convolutions and their transposed forms for the
        # input gradients, rewritten from the fp32 masters before every pass
        self.wb, self.wt, preps = {}, {}, []
        for name, kind, cin, cout in layer_specs(widths):
            if kind == "conv1":
                continue
            w = self.params[name + ".w"]
            self.wb[name] = torch.empty(w.shape, dtype=torch.bfloat16, device=device)
            tshape = (cin, 3, 3, cout) if kind == "conv3" else (cin, 2, 2, cout)
            self.wt[name] = torch.empty(tshape, dtype=torch.bfloat16, device=device)
            preps.append((w, name, W_CONV3 if kind == "conv3" else W_UP2, cout, cin))
        self._prep_train = _array(_WeightPrep, [
            _WeightPrep(w.data_ptr(), self.wb[n].data_ptr(), self.wt[n].data_ptr(), k, co, ci)
            for w, n, k, co, ci in preps])
        self._prep_infer = _array(_WeightPrep, [
            _WeightPrep(w.data_ptr(), self.wb[n].data_ptr(), None, k, co, ci)
            for w, n, k, co, ci in preps])
        # inference scale/shift from the running statistics
        self.scale = {n: torch.empty(P[n + ".gamma"].numel(), device=device) for n in self.bn_names}
        self.shift = {n: torch.empty(P[n + ".gamma"].numel(), device=device) for n in self.bn_names}
        self._bn = _array(_BnLayer, [
            _BnLayer(self.params[n + ".gamma"].numel(), self.batch_mr[n].data_ptr(),
                     self.running[n][0].data_ptr(), self.running[n][1].data_ptr(),
                     self.params[n + ".gamma"].data_ptr(), self.params[n + ".beta"].data_ptr(),
                     self.scale[n].data_ptr(), self.shift[n].data_ptr())
            for n in self.bn_names])

    def prepare_weights(self, with_transposed: bool = True):
        """Write the bf16 weights (and, for training, their transposed forms)
        from the current fp32 masters: one launch for all layers."""
        arr = self._prep_train if with_transposed else self._prep_infer
        _call("sil_unet_prep_weights", ctypes.cast(arr, ctypes.c_void_p), len(arr), _s())

    def forward(self, x: torch.Tensor, labels: torch.Tensor, with_logits: bool = True):
        """x: bf16 [N, H, W, 8]; labels: uint8 [N, H, W].  Returns (loss, logits);
        with_logits=False leaves the logits unwritten (an empty tensor), as
        the training step needs only the loss and its gradient.

        Starts a training step: the step's zeroed scratch (batch-norm sums and
        gradient accumulators) is taken from one pool cleared here, so the
        gradients of the previous step must have been consumed (optimizer step
        taken, zero_grad called) before the next forward."""
        self.pool.begin_step(x.device)
        self.prepare_weights(with_transposed=True)
        P = self.params
        skips = []
        h = x
        L = len(self.widths)
        # Every conv + BN + ReLU output has one consumer (the next conv, the
        # pooling layer, an up-convolution or the head): the consumer's
        # backward forms the layer's batch-norm sums (slot links).
        link = None  # the link of the layer that produced h

        def cbr(h, skip, n, in_slot):
            slot = _BnSlot()
            out = Conv3x3BNReLU.apply(h, skip, P[n + ".w"], P[n + ".gamma"], P[n + ".beta"],
                                      self.batch_mr[n], self.pool, self.wb[n], self.wt[n], slot,
                                      in_slot)
            return out, slot

        for i in range(L):
            name = f"enc{i}" if i < L - 1 else "mid"
            h, link = cbr(h, None, name + ".conv0", link)
            h, link = cbr(h, None, name + ".conv1", link)
            if i < L - 1:
                h, skip = MaxPool2.apply(h, link, self.pool)
                skips.append(skip)
                link = None
        for i in reversed(range(L - 1)):
            n = f"dec{i}.up"
            up = UpConv2.apply(h, P[n + ".w"], P[n + ".b"], self.pool, self.wb[n], self.wt[n],
                               link)
            h, link = cbr(up, skips[i], f"dec{i}.conv0", None)
            h, link = cbr(h, None, f"dec{i}.conv1", link)
        return HeadXent.apply(h, P["head.w"], P["head.b"], labels, self.pool, link, with_logits)

    def backward(self, loss: torch.Tensor):
        """loss.backward() with a seed gradient of 1 kept on the device, so that
        starting the backward pass launches no fill."""
        if getattr(self, "_one", None) is None or self._one.device != loss.device:
            self._one = torch.ones((), dtype=loss.dtype, device=loss.device)
        loss.backward(self._one)

    @torch.no_grad()
    def update_running_stats(self):
        """Exponential moving average of the last batch's statistics (biased
        batch variance recovered from rstd), all layers in one launch."""
        _call("sil_unet_bn_ema", ctypes.cast(self._bn, ctypes.c_void_p), len(self._bn),
              ctypes.c_float(self.momentum), ctypes.c_float(BN_EPS), _s())

    @torch.no_grad()
    def infer_logits(self, x: torch.Tensor) -> torch.Tensor:
        """Inference with the running statistics: fp32 logits [N, H, W, 3].  Every
        kernel treats pixels independently of the batch, so a chip's logits do
        not depend on the other chips of the batch."""
        P = self.params
        N, H, W, _ = x.shape
        dev = x.device
        self.prepare_weights(with_transposed=False)
        _call("sil_unet_bn_fold", ctypes.cast(self._bn, ctypes.c_void_p), len(self._bn),
              ctypes.c_float(BN_EPS), _s())

        def cbr(h, skip, n):
            Nn, Hh, Ww, c0 = h.shape
            c1 = 0 if skip is None else skip.shape[3]
            wb = self.wb[n]
            cout = wb.shape[0]
            out = torch.empty((Nn, Hh, Ww, cout), dtype=torch.bfloat16, device=dev)
            _call("sil_unet_conv3x3_affine_relu", _p(h), c0, _p(skip), c1, _p(wb),
                  _p(self.scale[n]), _p(self.shift[n]), _p(out), Nn, Hh, Ww, cout, _s())
            return out

        skips, h, L = [], x, len(self.widths)
        for i in range(L):
            name = f"enc{i}" if i < L - 1 else "mid"
            h = cbr(cbr(h, None, name + ".conv0"), None, name + ".conv1")
            if i < L - 1:
                h, skip = MaxPool2.apply(h)
                skips.append(skip)
        for i in reversed(range(L - 1)):
            n = f"dec{i}.up"
            up = UpConv2.apply(h, P[n + ".w"], P[n + ".b"], None, self.wb[n])
            h = cbr(cbr(up, skips[i], f"dec{i}.conv0"), None, f"dec{i}.conv1")
        C = h.shape[3]
        logits = torch.empty((N, H, W, 3), dtype=torch.float32, device=dev)
        _call("sil_unet_head", _p(h), _p(P["head.w"]), _p(P["head.b"]), _p(logits), N * H * W, C,
              _s())
        return logits

    def predict(self, x: torch.Tensor) -> torch.Tensor:
        """Class map [N, H, W] (uint8).  Uses batch statistics of `x`, as in training
        (a forward pass: it starts a step, see forward)."""
        N, H, W, _ = x.shape
        dummy = torch.zeros((N, H, W), dtype=torch.uint8, device=x.device)
        with torch.no_grad():
            _, logits = self.forward(x, dummy)
        out = torch.empty((N, H, W), dtype=torch.uint8, device=x.device)
        _call("sil_unet_argmax", _p(logits.contiguous()), _p(out), N * H * W, _s())
        return out


class Adam:
    """Adam on the model's fp32 master weights: every tensor with a gradient in
    one multi-tensor launch.  With use_device_step() the step number lives in
    device memory and is advanced by a kernel, so that a step captured in a
    graph counts correctly on every replay (self.t is then brought up to date
    by sync_step())."""

    def __init__(self, params: Dict[str, torch.Tensor], lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        self.params = params
        self.lr, self.b1, self.b2, self.eps = lr, betas[0], betas[1], eps
        self.m = {k: torch.zeros_like(v) for k, v in params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in params.items()}
        self.t = 0
        self.t_dev = None  # device int32: the number of the next step
        self._key = None
        self._arr = None

    def use_device_step(self):
        dev = next(iter(self.params.values())).device
        self.t_dev = torch.full((1,), self.t + 1, dtype=torch.int32, device=dev)

    def sync_step(self):
        if self.t_dev is not None:
            self.t = int(self.t_dev.item()) - 1

    @torch.no_grad()
    def step(self):
        self.t += 1
        items = []
        for k, p in self.params.items():
            if p.grad is None:
                continue
            g = p.grad if p.grad.is_contiguous() else p.grad.contiguous()
            items.append((p.data_ptr(), g.data_ptr(), self.m[k].data_ptr(),
                          self.v[k].data_ptr(), p.numel(), g))
        if not items:
            return
        key = tuple(it[:5] for it in items)
        if key != self._key:  # gradients usually sit at the same addresses every step
            self._arr = _array(_AdamTensor, [_AdamTensor(*it[:5]) for it in items])
            self._key = key
        _call("sil_unet_adam_multi", ctypes.cast(self._arr, ctypes.c_void_p), len(self._arr),
              ctypes.c_float(self.lr), ctypes.c_float(self.b1), ctypes.c_float(self.b2),
              ctypes.c_float(self.eps), self.t, _p(self.t_dev), _s())
        if self.t_dev is not None:
            _call("sil_unet_counter_add", _p(self.t_dev), 1, _s())

    def zero_grad(self):
        for p in self.params.values():
            p.grad = None


class CapturedStep:
    """One training step (forward, backward, Adam, running statistics) recorded
    once in a HIP graph (torch.cuda.graph over the library's launches) and
    replayed: no host work and no launch gaps per step.  The batch goes through
    static input tensors; the model's buffers, the step's zeroed scratch and
    the optimizer's step counter stay at the addresses recorded.  Call after at
    least one eager step (which sizes the scratch pool), with no autograd graph
    of an earlier step still alive (drop its loss tensor first: its gradient
    accumulators belong to the stream it ran on).  Recording launches nothing;
    every replay is one training step."""

    def __init__(self, model: "UNet", opt: Adam, x: torch.Tensor, labels: torch.Tensor):
        self.model, self.opt = model, opt
        self.x = x.clone()
        self.labels = labels.clone()
        if opt.t_dev is None:
            opt.use_device_step()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            opt.zero_grad()
            self.loss, _ = model.forward(self.x, self.labels, with_logits=False)
            model.backward(self.loss)
            opt.step()
            model.update_running_stats()
        opt.zero_grad()
        opt.t -= 1  # recording counted a step on the host that did not run

    def __call__(self, x: torch.Tensor, labels: torch.Tensor) -> torch.Tensor:
        """Copy the batch in, replay; returns the (static) loss tensor."""
        self.x.copy_(x)
        self.labels.copy_(labels)
        self.graph.replay()
        self.opt.t += 1
        return self.loss


def chips_input(scene: torch.Tensor, origins: torch.Tensor, chip: int = 256,
                refl_max: float = 10000.0, out: torch.Tensor = None) -> torch.Tensor:
    """bf16 [n, chip, chip, 8] network input from a [3, H, W] int16/uint16
    scene for the chip origins [n, 2] (int32, device), written to `out` when
    given (a contiguous [n, chip, chip, 8] bf16 tensor, e.g. a slice of a
    batch shared by several scenes)."""
    _, H, pitch = scene.shape
    n = origins.shape[0]
    if out is None:
        out = torch.empty((n, chip, chip, IN_CH), dtype=torch.bfloat16, device=scene.device)
    elif out.shape != (n, chip, chip, IN_CH) or out.dtype != torch.bfloat16 \
            or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous bf16 [{n}, {chip}, {chip}, {IN_CH}] tensor")
    _call("sil_unet_chips_input", _p(scene), H, pitch, pitch, _p(origins.contiguous()), n, chip,
          ctypes.c_float(1.0 / refl_max), _p(out), _s())
    return out


def scatter_argmax(logits: torch.Tensor, origins: torch.Tensor, labels: torch.Tensor, H: int,
                   W: int):
    """Class map of chips written into a scene label plane [H, >=W] (uint8)."""
    n, chip = logits.shape[0], logits.shape[1]
    _call("sil_unet_scatter_argmax", _p(logits.contiguous()), _p(origins.contiguous()), n, chip,
          _p(labels), H, W, labels.stride(0), _s())


# ---- checkpoints -------------------------------------------------------------------

def save_checkpoint(path: str, model: "UNet", opt: "Adam" = None, extra: Dict[str, int] = None):
    """Write the model (fp32 master weights, running batch-norm statistics) and,
    when given, the Adam state (moments and step count) to a safetensors file.
    Integer metadata (e.g. the training step and the sampler seed) goes in
    ``extra``.  The file's metadata records the widths and a SHA-256 over all
    tensors, which load_checkpoint verifies."""
    import hashlib
    from safetensors.torch import save_file
    tensors = {}
    for k, v in model.params.items():
        tensors["param." + k] = v.detach().contiguous().cpu()
    for n, (rm, rv) in model.running.items():
        tensors["running_mean." + n] = rm.detach().contiguous().cpu()
        tensors["running_var." + n] = rv.detach().contiguous().cpu()
    meta = {"widths": ",".join(str(w) for w in model.widths)}
    if opt is not None:
        for k in opt.m:
            tensors["adam_m." + k] = opt.m[k].detach().contiguous().cpu()
            tensors["adam_v." + k] = opt.v[k].detach().contiguous().cpu()
        meta["adam_t"] = str(opt.t)
        meta["adam_lr"] = repr(opt.lr)
    for k, v in (extra or {}).items():
        meta["extra." + k] = str(int(v))
    h = hashlib.sha256()
    for k in sorted(tensors):
        h.update(k.encode())
        h.update(tensors[k].numpy().tobytes())
    meta["sha256"] = h.hexdigest()
    save_file(tensors, path, metadata=meta)


def load_checkpoint(path: str, device="cuda", lr: float = None):
    """Read a file written by save_checkpoint: returns (model, opt or None,
    extra).  Raises ValueError when the tensors do not match the recorded
    SHA-256."""
    import hashlib
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        meta = f.metadata()
        tensors = {k: f.get_tensor(k) for k in f.keys()}
    h = hashlib.sha256()
    for k in sorted(tensors):
        h.update(k.encode())
        h.update(tensors[k].numpy().tobytes())
    if h.hexdigest() != meta.get("sha256"):
        raise ValueError(f"{path}: checkpoint hash mismatch")
    widths = tuple(int(w) for w in meta["widths"].split(","))
    model = UNet(widths, device=device)
    with torch.no_grad():
        for k, v in model.params.items():
            v.copy_(tensors["param." + k].to(device))
        for n, (rm, rv) in model.running.items():
            rm.copy_(tensors["running_mean." + n].to(device))
            rv.copy_(tensors["running_var." + n].to(device))
    opt = None
    if "adam_t" in meta:
        opt = Adam(model.params, lr=float(meta["adam_lr"]) if lr is None else lr)
        for k in opt.m:
            opt.m[k].copy_(tensors["adam_m." + k].to(device))
            opt.v[k].copy_(tensors["adam_v." + k].to(device))
        opt.t = int(meta["adam_t"])
    extra = {k[len("extra."):]: int(v) for k, v in meta.items() if k.startswith("extra.")}
    return model, opt, extra
