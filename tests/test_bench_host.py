"""Host-side pieces of bench.py (no GPU): the one-GPU contract, the issue
ceiling arithmetic, and the committed counter summaries it reads."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_issue_ceiling_adds_each_class_at_its_own_rate():
    import bench
    rates = {k: {"rate": 1.0} for k in bench.STEP_CLASSES}
    for k in bench.FULL_RATE_FORMS:
        rates[k] = {"rate": 2.0}
    rates[bench.FULL_RATE_FORMS[0]] = {"rate": 4.0}     # the fastest full-rate form is used
    want = sum(n / (4.0 if k == "full_rate" else 1.0) for k, n in bench.STEP_CLASSES.items())
    assert bench.issue_ceiling_step_time(rates) == pytest.approx(want)


def test_profile_values_are_read_only_for_the_current_kernel_sources(tmp_path):
    import bench
    good = tmp_path / "good.txt"
    good.write_text(f"# comment: ignored\nkernel_hash: {bench.kernel_hash()}\nfigure: 12.5\n")
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_hash: 0000000000000000\nfigure: 12.5\n")
    assert bench.profile_value(str(good), "figure") == 12.5
    assert bench.profile_value(str(stale), "figure") is None
    assert bench.profile_value(str(good), "missing") is None
    assert bench.profile_value(str(tmp_path / "absent.txt"), "figure") is None


def test_committed_walk_counters_match_the_kernel_sources():
    """The traffic and FP32 figures of the bench line come from committed
    rocprofv3 summaries; they are used only while the walk's sources hash to
    the value recorded with them, so a kernel change needs the counters
    taken again."""
    import bench
    assert bench.measured_traffic() is not None
    assert bench.profile_value(os.path.join(ROOT, "profiles", "walk_two_species_500_valu_counters.txt"),
                               "fp32_flop_per_photon_step") is not None
