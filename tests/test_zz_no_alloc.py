"""GPU test of sil_label_ex_noalloc, the general labeller whose workspace is
the library's own per-device array: two calls in a row, the second on a
smaller scene, each bit-identical to sil_label_ex with a caller workspace,
for chip-level full-HSV limits and for the whole scene as one filter unit
with the filtered colour image; scenes needing more workspace than the array
holds are refused before anything is enqueued."""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

LIMITS = dict(lo=[[0, 40, 0], [20, 0, 60], [100, 10, 150]],
              hi=[[90, 255, 120], [179, 200, 220], [170, 255, 255]])


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


def _scene(H, W, seed):
    spec = synth.SceneSpec(H, W, seed, "u16", synth.blobs_for_coverage(H, W, seed, 1, 2, 0.10),
                           synth.blobs_for_coverage(H, W, seed, 2, 1, 0.05))
    return torch.from_numpy(synth.generate(spec).view(np.int16)).cuda()


@pytest.mark.parametrize("name,kw,rgb", [("full-HSV chip 256", dict(chip=256, **LIMITS), False),
                                         ("scene as one unit", dict(chip=1 << 20), True)])
def test_noalloc_equals_workspace_calls(sil, name, kw, rgb):
    p = sil.Params(dtype=sil.U16, **kw)
    for H, W, seed in ((2048, 1536, 91), (700, 900, 92)):  # the second call is smaller
        _say(f"case noalloc {name} {H}x{W}")
        s = _scene(H, W, seed)
        ref = sil.label_ex(s, p, rgb=rgb, chips=True)
        got = sil.label_ex(s, p, rgb=rgb, chips=True, noalloc=True)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(got[k], ref[k]), f"{name} {H}x{W}: {k} differs"


def test_noalloc_refuses_scenes_beyond_its_array(sil):
    import ctypes
    p = sil.Params(dtype=sil.U16, chip=256)
    assert sil.workspace_bytes(8192, 8192, p) > (32 << 20)
    s = torch.zeros((3, 8, 8), dtype=torch.int16, device="cuda")
    masks = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    pc = p.to_c()
    # sizes are checked before anything is enqueued: neither buffer is touched
    rc = sil.lib().sil_label_ex_noalloc(
        ctypes.c_void_p(s.data_ptr()), 3, (ctypes.c_int32 * 3)(0, 1, 2), 8192, 8192, 8192,
        ctypes.byref(pc), ctypes.c_void_p(masks.data_ptr()), 8192, None, None, 0, None, None)
    assert rc == sil.EUNSUPPORTED
