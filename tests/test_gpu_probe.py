"""The latency probes behind the decode bound run, and give plausible numbers."""
import pytest

import paper_2207_05152_amd as dl
from gpu_util import dev, say  # noqa: F401

pytestmark = pytest.mark.gpu


def test_latency_probe(dev):
    say("latency probe")
    r = dl.dlic_latency_probe()
    assert 1000.0 < r["shader_clock_mhz"] < 3000.0
    for name in dl.PROBE_NAMES:
        assert 0.5 < r[name] < 20000.0, (name, r[name])
    # a chain of FP32 FMAs cannot beat one issue per link, and a hand-off
    # through device memory is slower than one through LDS
    assert r["fma_f32"] >= 1.0
    assert r["global_flag_handoff"] > r["lds_flag_handoff"]
