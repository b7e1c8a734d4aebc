"""Frozen seeded inputs (CPU): shapes, ranges and SHA-256 digests."""
import hashlib

import numpy as np

import synth


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def test_shapes_and_types():
    im = synth.synth_image(48, 80, 3)
    assert im.shape == (48, 80) and im.dtype == np.uint8
    ph = synth.mri_phantom(2000)
    assert ph.shape == (256, 256) and ph.dtype == np.uint8
    w = synth.xavier_mlp((12, 64, 64, 15), 3)
    assert w["W1"].shape == (64, 12) and w["W2"].shape == (64, 64) and w["W3"].shape == (15, 64)
    assert all(v.dtype == np.float32 for v in w.values())
    lim = np.sqrt(6.0 / (64 + 64))
    assert np.abs(w["W2"]).max() <= lim
    idx = synth.train_indices(0, 1000, 256, 256, 256)
    assert idx.shape == (1000, 3) and idx.min() >= 0 and idx.max() < 256


def test_deterministic():
    assert np.array_equal(synth.synth_image(30, 20, 5), synth.synth_image(30, 20, 5))
    assert not np.array_equal(synth.synth_image(30, 20, 5), synth.synth_image(30, 20, 6))


def test_tables_valid():
    t = synth.random_tables(50, 0)
    assert (t[:, 0] == 0).all() and (t[:, -1] == 65536).all() and (np.diff(t.astype(np.int64), axis=1) >= 1).all()


def test_frozen_digests():
    # Digests taken when the recipes were fixed; a change means every stored
    # expectation built on these inputs must be regenerated.
    cat = lambda w: np.concatenate([v.ravel() for k, v in sorted(w.items())])
    assert _sha(synth.synth_image(64, 64, 42)) == "9b736e28766c067d"
    assert _sha(cat(synth.xavier_mlp((12, 32, 32, 15), 7))) == "e099f6af56746afa"
    assert _sha(cat(synth.xavier_mlp((12, 64, 64, 15), 3))) == "95746706a4c78c26"
    assert _sha(synth.mri_phantom(2000)) == "e9ce845f50d81e98"
    assert _sha(synth.mri_volume(2024)) == "0f17a7e3c311f383"
    v12 = synth.mri_volume(5, 3, 32, bits=12)
    assert v12.dtype == np.uint16 and v12.max() < 4096
    assert _sha(v12) == "df3185f795d56173"
