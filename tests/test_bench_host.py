"""Host-side logic of bench.py (no GPU): the one-GPU guard, the counter-summary lookup that
supplies the roofline's measured traffic, and the host description of the CPU baseline."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SOURCES = ("nb_forces.hip", "nb_internal.h", "nb_erfc_coeffs.h", "nb_pair_common.h")


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""        # no JSON line


def _fake_root(tmp_path, profile_text, tamper=False):
    """A tree with the kernel sources (optionally one byte changed) and one counter summary."""
    csrc = tmp_path / "paper_2006_09167_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2006_09167_amd", "csrc", f), csrc / f)
    if tamper:
        with open(csrc / "nb_internal.h", "a") as fh:
            fh.write("\n")
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k_nb_fwd_water96k_ewald_counters.txt").write_text(profile_text)
    return str(tmp_path)


def test_traffic_is_read_for_the_summarised_shapes_only(monkeypatch):
    path = os.path.join(ROOT, "profiles", "k_nb_fwd_water96k_ewald_counters.txt")
    with open(path) as fh:
        lines = [l for l in fh.read().splitlines() if l.strip().startswith("HBM traffic")]
    assert lines, "the committed summary has no traffic line"
    for line in lines:
        width = int(line.split("scaled, ")[1].split(" entries")[0])
        mode = {"persistent rounds": "persist", "XCD-contiguous": "xcd", "static": "static",
                "balanced runs + dynamic tail": "queue",
                "equal-cost runs": "balanced"}[line.split("per item, ")[1].split(")")[0]]
        got = bench.measured_traffic("water96k_ewald", {"item_width": width, "mode": mode})
        if got is None:
            pytest.skip("kernel sources changed since the counters were taken")
        assert got == pytest.approx(float(line.split()[-2]) * 1e6)
    # a shape the summary does not cover, and a workload without a summary
    assert bench.measured_traffic("water96k_ewald", {"item_width": 17, "mode": "static"}) is None
    assert bench.measured_traffic("water1500k_ewald", {"item_width": 36, "mode": "persist"}) is None


def test_traffic_needs_the_hash_of_the_current_sources(tmp_path, monkeypatch):
    import hashlib
    src = b"".join(open(os.path.join(ROOT, "paper_2006_09167_amd", "csrc", f), "rb").read()
                   for f in SOURCES)
    h = hashlib.sha256(src).hexdigest()[:16]
    text = ("sources %s\nHBM traffic (MB = 1e6 B, scaled, 24 entries per item, static)"
            "    12.50 MB\n" % h)
    monkeypatch.setattr(bench, "ROOT", _fake_root(tmp_path / "a", text))
    assert bench.measured_traffic("water96k_ewald",
                                  {"item_width": 24, "mode": "static"}) == pytest.approx(12.5e6)
    assert bench.measured_traffic("water96k_ewald", {"item_width": 24, "mode": "xcd"}) is None
    # the same summary beside sources that differ from the ones it was taken on
    monkeypatch.setattr(bench, "ROOT", _fake_root(tmp_path / "b", text, tamper=True))
    assert bench.measured_traffic("water96k_ewald", {"item_width": 24, "mode": "static"}) is None


def test_host_info_reports_the_cpus():
    info = bench.host_info()
    assert info["nproc"] == os.cpu_count() and info["nproc"] >= 1
    assert info["model"] is None or isinstance(info["model"], str)


def test_flop_counts_match_their_itemisation():
    # the per-slot counts the roofline credits, summed from the items their comment lists
    common = 3 + 5 + 1 + 1 + 5 + 1 + 9
    ewald = 1 + 3 + 14 + 1 + 1 + 1 + 1 + 3 + 3 + 9
    rf = 5 + 14
    assert bench.FLOP_PER_PAIR == {"ewald": common + ewald, "rf": common + rf}
    assert bench.FLOP_PER_PAIR_LJ_FORCE == common - 1 + 1
