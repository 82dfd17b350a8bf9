"""GPU tests of sil_render_rgb (class-id plane -> the paper's colours) against
the oracle's rendering, bit for bit: random ids (the three classes and every
other byte value), ragged widths and odd pitches (the byte path), padded
colour rows (left untouched), a labelled full 10980 x 10980 tile, and the
argument errors."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from oracle import sil_ref as R
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sil():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_13135_amd import sil as S
    S.lib()
    return S


def _ids(rng, H, pitch):
    lab = rng.integers(0, 3, size=(H, pitch)).astype(np.uint8)
    other = rng.random((H, pitch)) < 0.1
    lab[other] = rng.integers(3, 256, size=int(other.sum())).astype(np.uint8)
    return lab


@pytest.mark.parametrize("H,W,pitch,rgb_pad", [(1, 1, 1, 0), (2, 3, 3, 0), (5, 7, 9, 5),
                                               (64, 1001, 1024, 0), (33, 4096, 4100, 12),
                                               (17, 998, 1000, 3)])
def test_render_matches_oracle(sil, H, W, pitch, rgb_pad):
    _say(f"case render H={H} W={W} pitch={pitch} rgb_pad={rgb_pad}")
    rng = np.random.default_rng(H * 7 + W)
    lab = _ids(rng, H, pitch)
    want = R.render_rgb(lab, W=W)
    labc = torch.from_numpy(lab).cuda()
    # colour rows of 3 (W + rgb_pad) bytes, pre-filled, so that the padding can be checked
    buf = torch.full((H, W + rgb_pad, 3), 77, dtype=torch.uint8, device="cuda")
    out = sil.render_rgb(labc, W=W, out=buf[:, :W])
    torch.cuda.synchronize()
    assert out.data_ptr() == buf.data_ptr()
    got = buf.cpu().numpy()
    assert (got[:, :W] == want).all()
    assert (got[:, W:] == 77).all()


def test_render_of_labelled_full_tile(sil):
    """The labels of the full tile (the benchmark's workload) rendered on the
    GPU equal the oracle's rendering of the same labels."""
    _say("case render full tile: generating")
    s = synth.generate(synth.config_tile())
    t = torch.from_numpy(s.view(np.int16)).cuda()
    _say("case render full tile: label and render")
    labels, _ = sil.label(t, sil.Params(dtype=sil.U16))
    rgb = sil.render_rgb(labels, W=s.shape[2])
    torch.cuda.synchronize()
    lab = labels.cpu().numpy()
    _say("case render full tile: oracle")
    want = R.render_rgb(lab, W=s.shape[2])
    assert (rgb.cpu().numpy() == want).all()


def test_render_argument_errors(sil):
    lab = torch.zeros((4, 8), dtype=torch.uint8, device="cuda")
    rgb = torch.empty((4, 8, 3), dtype=torch.uint8, device="cuda")
    L = sil.lib()
    p, q, st = ctypes.c_void_p(lab.data_ptr()), ctypes.c_void_p(rgb.data_ptr()), None
    assert L.sil_render_rgb(None, 4, 8, 8, q, 24, st) == sil.EINVAL
    assert L.sil_render_rgb(p, 0, 8, 8, q, 24, st) == sil.EINVAL
    assert L.sil_render_rgb(p, 4, 8, 7, q, 24, st) == sil.EINVAL   # label pitch < W
    assert L.sil_render_rgb(p, 4, 8, 8, q, 23, st) == sil.EINVAL   # colour pitch < 3 W
    assert L.sil_render_rgb(p, 4, 8, 8, q, 24, st) == sil.OK
    torch.cuda.synchronize()
