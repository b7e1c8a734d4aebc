"""The decoder's waves hand data to each other through LDS counters and, between row
groups, through device memory.  With seeded pauses injected at the coder, the density
waves and the courier (the dlic_set_decode_delays hook), those hand-offs meet in other
orders; every decode must still return the encoded image bit for bit."""
import numpy as np
import pytest
import torch

import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture
def delays():
    yield dl.dlic_set_decode_delays
    dl.dlic_set_decode_delays(0, 0)


@pytest.mark.parametrize("h,w,width,G,L", [
    (96, 160, 64, 4, 4),      # 16 coder lanes per pixel, 4-pixel net
    (120, 90, 64, 2, 32),     # 2 lanes per pixel
    (64, 200, 128, 16, 4),    # one sub-round per step, 128-wide 4-pixel net
    (70, 64, 32, 1, 64),      # one lane per pixel, 64 lanes
])
@pytest.mark.parametrize("seed,max_cycles", [(1, 3000), (2, 20000)])
def test_round_trip_under_injected_delays(dev, delays, h, w, width, G, L, seed, max_cycles):
    img = synth.synth_image(h, w, 17 + seed)
    m = dl.Model(synth.xavier_mlp((12, width, width, 15), 3), dev)
    coder = dl.dlic_coder(G, L)
    bits = dl.encode(to_dev(img, dev), m, coder)
    delays(seed, max_cycles)
    say("delays", h, w, width, G, L, seed, max_cycles)
    dec, st = dl.decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0
    assert np.array_equal(dec.cpu().numpy(), img)


def test_batch_under_injected_delays(dev, delays):
    m = dl.Model(synth.xavier_mlp((12, 64, 64, 15), 3), dev, dtype="bf16")
    sizes = [(60, 80), (33, 100), (90, 40), (16, 16)]
    imgs = [synth.synth_image(h, w, 40 + i) for i, (h, w) in enumerate(sizes)]
    b = dl.Batch(m, sizes, coders=[(3, 4), (2, 32), (4, 16), (1, 4)])
    b.load(imgs)
    b.encode()
    torch.cuda.synchronize()
    delays(5, 8000)
    say("batch delays")
    b.decode()
    torch.cuda.synchronize()
    assert np.array_equal(b.status.cpu().numpy(), np.zeros(len(sizes)))
    for i, img in enumerate(imgs):
        assert np.array_equal(b.image(i).cpu().numpy(), img), i
    b.close()


@pytest.mark.parametrize("seed,max_cycles", [(1, 3000), (2, 20000)])
def test_softmax_and_volume_decoders_under_injected_delays(dev, delays, seed, max_cycles):
    # the six-layer decoder hands tables and pixels between workgroups through per-row
    # step counters; pauses at the tile's wait, before its tables are published, at the
    # coder's wait and before its pixels are published reorder those hand-offs
    layers = synth.xavier_deep(64, 5)
    m = dl.DeepModel(layers, dev)
    img = synth.synth_image(48, 70, 3 + seed)
    bits = dl.deep_encode(to_dev(img, dev), m, dl.dlic_coder(3, 4))
    m3 = dl.DeepModel(synth.xavier_deep(64, 6, k_in=21), dev)
    vol = synth.mri_volume(30 + seed, 4, 24)[:, :, :20]
    vbits = dl.volume_encode(to_dev(vol, dev), m3, dl.dlic_coder(2, 4), 1)
    torch.cuda.synchronize()
    delays(seed, max_cycles)
    say("deep delays", seed, max_cycles)
    dec, st = dl.deep_decode(bits, m, check=False)
    vdec, vst = dl.volume_decode(vbits, m3, check=False)
    torch.cuda.synchronize()
    assert st == 0 and np.array_equal(dec.cpu().numpy(), img)
    assert vst == 0 and np.array_equal(vdec.cpu().numpy(), vol)
