"""Host-side checks of bench.py: the one-GPU guard and the paper's timing context."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 1" in r.stderr
    assert r.stdout == ""


def test_paper_context_rates():
    # Section IV-D, Table III: a 256x256x35 scan coded completely in 0.3374 s
    # is 2 293 760 px / 0.3374 s = 6.798 MPix/s; the 92M-parameter net's
    # 7.1203 s is 0.322 MPix/s
    mri = bench.PAPER_CONTEXT["mri_estimated"]
    assert len(mri["params"]) == len(mri["first_frame_s"]) == len(mri["complete_s"]) == 5
    assert mri["complete_mpix_s"][0] == pytest.approx(6.798, abs=1e-3)
    assert mri["complete_mpix_s"][-1] == pytest.approx(0.322, abs=1e-3)
    # the first frame is ready before the scan is complete, and larger nets are slower
    assert all(a < b for a, b in zip(mri["first_frame_s"], mri["complete_s"]))
    assert mri["complete_s"] == sorted(mri["complete_s"])


def test_source_digest_is_stable():
    a, b = bench.kernel_sources_sha256(), bench.kernel_sources_sha256()
    assert a == b and len(a) == 64


PROBE = {"fma_f32": 5.6, "mfma_4x4x1_f32": 12.6, "mfma_16x16x4_f32": 32.4, "lds_store_load": 118.0,
         "lds_load": 72.0, "lds_flag_handoff": 234.0, "dpp_reduce16": 54.0, "expf": 75.0,
         "rans_update": 39.0, "ballot_popcount": 34.0, "global_flag_handoff": 1760.0,
         "readlane": 31.0, "shader_clock_mhz": 2400.0}


def test_step_chain_by_hand():
    dens, coder, parts = bench.step_chain_cycles(PROBE, 64)
    f = 5.6
    table = 15 * f + 72.0
    want_dens = ((118 + 3 * f) + 4 * f + (118 + 64 * f + f) + (118 + 19 * f)
                 + (11 * f + 75) + (118 + table))
    want_coder = (f + 54) + table + (f + 54) + (39 + 34 + 31 + f)
    assert dens == pytest.approx(want_dens)
    assert coder == pytest.approx(want_coder)
    assert sum(parts.values()) == pytest.approx(dens + coder)
    # 32 wide: layer 3 is one chain over all 32 inputs
    d32, _, _ = bench.step_chain_cycles(PROBE, 32)
    assert d32 == pytest.approx(want_dens - 64 * f + 32 * f - 19 * f + 32 * f)


def test_latency_bound_takes_the_longer_chain():
    dens, coder, _ = bench.step_chain_cycles(PROBE, 64)
    T = 2048 + 3 * 1536 - 3
    # 64 groups of 4 lanes: 24 rows per group, 6 rows per lane and step
    ms, d = bench.decode_latency_bound_ms(PROBE, 1536, 2048, 64, 4, 64)
    assert d["rows_per_lane_per_step"] == 6 and d["steps"] == T
    assert d["per_step_cycles"] == pytest.approx(max(6 * coder, dens + coder))
    assert ms == pytest.approx((T * d["per_step_cycles"] + 63 * (1760 - 118)) / 2.4e6)
    # one lane per row: the density-coder loop of one step bounds it
    ms1, d1 = bench.decode_latency_bound_ms(PROBE, 1536, 2048, 384, 4, 64)
    assert d1["rows_per_lane_per_step"] == 1
    assert d1["per_step_cycles"] == pytest.approx(dens + coder)


def test_latency_bound_with_strips():
    dens, coder, _ = bench.step_chain_cycles(PROBE, 64)
    T = 2048 + 3 * 1536 - 3
    # 64 groups of 4 lanes, 2 strips each: 12 rows per strip, 3 rows per lane and step,
    # and 127 strip boundaries between workgroups
    ms, d = bench.decode_latency_bound_ms(PROBE, 1536, 2048, 64, 4, 64, 2)
    assert d["rows_per_lane_per_step"] == 3
    assert d["per_step_cycles"] == pytest.approx(max(3 * coder, dens + coder))
    assert ms == pytest.approx((T * d["per_step_cycles"] + 127 * (1760 - 118)) / 2.4e6)


def test_schedule_bound_with_strips_by_brute_force():
    h, w, G, S = 24, 10, 2, 2
    rows = [(b * h) // (G * S) for b in range(G * S + 1)]
    T = w + 3 * h - 3
    want = 0
    for t in range(T):
        worst = 0
        for g in range(G):
            n = sum(1 for b in range(g, G * S, G) for y in range(rows[b], rows[b + 1])
                    if 0 <= t - 3 * y < w)
            worst = max(worst, n)
        want += worst
    assert bench.schedule_bound_px(h, w, G, S) == want
    assert bench.schedule_bound_px(h, w, G, 1) >= want
