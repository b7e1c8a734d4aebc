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
