"""Edge cases of the decode path on the GPU: the bounded wait for the group
above (forced from the host with a one-poll spin limit), the largest group
count (more workgroups than compute units), and very wide images."""
import numpy as np
import pytest
import torch

import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _roundtrip(dev, img, width, coder):
    m = dl.Model(synth.xavier_mlp((12, width, width, 15), 3), dev)
    bits = dl.encode(to_dev(img, dev), m, coder)
    out, st = dl.decode(bits, m, check=False)
    torch.cuda.synchronize()
    return m, bits, out.cpu().numpy(), st


@pytest.mark.parametrize("L", [8, 4])
def test_timeout_of_upstream_wait_is_reported_and_recoverable(dev, L):
    img = synth.synth_image(96, 300, 5)
    coder = dl.dlic_coder(4, L)
    m = dl.Model(synth.xavier_mlp((12, 32, 32, 15), 3), dev)
    bits = dl.encode(to_dev(img, dev), m, coder)
    torch.cuda.synchronize()
    say("decode with a one-poll spin limit")
    dl.dlic_set_spin_limit(1)
    try:
        _, st = dl.decode(bits, m, check=False)
        torch.cuda.synchronize()
    finally:
        dl.dlic_set_spin_limit(1 << 22)
    # groups 1..3 start by waiting for the group above: one poll cannot see
    # its records, so the wait gives up, says so, and the grid still drains
    assert st == dl.DLIC_ERR_TIMEOUT
    say("decode again with the default limit")
    out, st = dl.decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == dl.DLIC_OK and np.array_equal(out.cpu().numpy(), img)


def test_most_groups_more_than_compute_units(dev):
    # 1024 groups of 2 rows: four times the CU count, so later groups start
    # only as earlier ones finish; each waits only for the one before it
    h, w = 2048, 40
    img = synth.synth_image(h, w, 77)
    say("1024 groups")
    _, bits, out, st = _roundtrip(dev, img, 32, dl.dlic_coder(1024, 2))
    assert st == dl.DLIC_OK and np.array_equal(out, img)
    hd = dl.dlic_peek_header(bits[:dl.HEADER_BYTES].cpu().numpy().tobytes())
    assert hd["coder"].groups == 1024


@pytest.mark.parametrize("h,w,G,L", [(3, 70000, 1, 4), (256, 1, 1, 64), (64, 4099, 2, 64)])
def test_extreme_shapes(dev, h, w, G, L):
    img = synth.synth_image(h, w, h + w)
    say("shape", h, w, G, L)
    _, _, out, st = _roundtrip(dev, img, 64, dl.dlic_coder(G, L))
    assert st == dl.DLIC_OK and np.array_equal(out, img)
