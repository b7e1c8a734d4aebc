"""The decode entry point that allocates nothing (a fixed workspace array in the library)
against dlic_decode on the same streams: same pixels and status, on two calls in a row, the
second with a smaller image (and the first with two row strips per group), and a layout
beyond the array's limit refused."""
import numpy as np
import pytest
import torch

import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _decode_both(dev, bits, model, h, w, coder):
    ref = torch.full((h, w), 7, dtype=torch.uint8, device=dev)
    st_ref = torch.full((1,), -1, dtype=torch.int32, device=dev)
    wsb = dl.dlic_decode_workspace(h, w, coder)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    dl.dlic_decode(model.c, coder, bits, bits.numel(), ref, h, w, st_ref, ws, wsb)
    got = torch.full((h, w), 9, dtype=torch.uint8, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    dl.dlic_decode_noalloc(model.c, coder, bits, bits.numel(), got, h, w, st)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), int(st_ref.item()), got.cpu().numpy(), int(st.item())


@pytest.mark.parametrize("dtype,width", [("fp32", 64), ("bf16", 128)])
def test_noalloc_decode_matches_decode_twice(dev, dtype, width):
    model = dl.Model(synth.xavier_mlp((12, width, width, 15), 3), dev, dtype=dtype)
    # first a large image (2048x1536, 64 groups x 4 lanes, two row strips per group: one
    # record row per strip), then a smaller one with one strip: the second call must not
    # see the first's records (the array keeps the last call's contents)
    for h, w, G, L, S, seed in ((1536, 2048, 64, 4, 2, 1), (300, 257, 6, 32, 1, 2)):
        img = synth.synth_image(h, w, seed)
        coder = dl.dlic_coder(G, L, S)
        say("noalloc decode", dtype, width, h, w, G, L, S)
        bits = dl.encode(to_dev(img, dev), model, coder)
        ref, st_ref, got, st = _decode_both(dev, bits, model, h, w, coder)
        assert st_ref == 0 and st == 0, (st_ref, st)
        assert np.array_equal(ref, img)
        assert np.array_equal(got, ref)


def test_noalloc_decode_reports_corruption_like_decode(dev):
    model = dl.Model(synth.xavier_mlp((12, 32, 32, 15), 7), dev)
    img = synth.synth_image(64, 96, 5)
    coder = dl.dlic_coder(2, 32)
    bits = dl.encode(to_dev(img, dev), model, coder)
    bad = bits.clone()
    bad[bad.numel() // 2] ^= 0x5A
    say("noalloc corrupt")
    _, st_ref, _, st = _decode_both(dev, bad, model, 64, 96, coder)
    assert st_ref == st and st != 0


def test_noalloc_decode_limit(dev):
    model = dl.Model(synth.xavier_mlp((12, 32, 32, 15), 7), dev)
    limit = dl.DECODE_NOALLOC_BYTES
    assert limit == 8 << 20
    # 1024 groups of 4 rows over a 4096 x 8192 image: far beyond the array
    coder = dl.dlic_coder(1024, 4)
    assert dl.dlic_decode_workspace(4096, 8192, coder) > limit
    dummy = torch.zeros(64, dtype=torch.uint8, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    with pytest.raises(dl.DlicError) as e:
        dl.dlic_decode_noalloc(model.c, coder, dummy, 64, dummy, 4096, 8192, st)
    assert e.value.status == dl.DLIC_ERR_CAPACITY
