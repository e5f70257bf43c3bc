"""CPU: bench.py's host logic -- the one-GPU contract, the roofline
arithmetic of the dominant pass kernel and the guard that drops the stored
HBM-traffic figure once the kernel sources differ from those it was measured
on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _acc(t_ph, t_e, n_ph, n_e, events, steps, t_round=0.0, n_round=0, interactions=0):
    a = bench.Acc()
    a.add({"t_photon_pass_s": t_ph, "t_electron_pass_s": t_e, "n_photon_launches": n_ph, "n_electron_launches": n_e,
           "t_round_s": t_round, "n_round_launches": n_round, "n_e_steps": steps, "n_photon_events": events,
           "n_photon_interactions": interactions, "ledger_residual_lsb": 0, "n_hist": 1})
    return a


def test_roofline_of_the_dominant_kernel():
    # electron pass dominant: 10 launches of 2 ms, 1e8 steps -> 1e7 steps per launch
    r = bench.roofline(_acc(0.005, 0.020, 10, 10, 2e8, 1e8), "x")
    assert r["kernel"] == "k_electron_pass"
    assert r["avg_launch_ms"] == pytest.approx(2.0)
    assert r["achieved"] == pytest.approx(1e7 * bench.OPS_PER_E_STEP / 2e-3 / 1e12)
    assert r["peak"] == pytest.approx(256 * 64 * 2.4e9 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["traffic"] is None          # only the water workload carries the measured bytes
    assert r["k_photon_pass"]["achieved"] == pytest.approx(2e8 * bench.OPS_PER_PH_EVENT / 0.005 / 1e12)
    # photon pass dominant: flights plus real interactions
    r = bench.roofline(_acc(0.030, 0.020, 10, 10, 2e8, 1e8, interactions=5e7), "x")
    assert r["kernel"] == "k_photon_pass"
    assert r["achieved"] == pytest.approx((2e8 * bench.OPS_PER_PH_EVENT + 5e7 * bench.OPS_PER_PH_INTERACTION)
                                          / 10 / 3e-3 / 1e12)
    # the persistent round kernel, when it holds most of the time, counts both types' work
    r = bench.roofline(_acc(0.001, 0.001, 1, 1, 2e8, 1e8, t_round=0.05, n_round=5), "x")
    assert r["kernel"] == "k_round"
    assert r["achieved"] == pytest.approx((1e8 * bench.OPS_PER_E_STEP + 2e8 * bench.OPS_PER_PH_EVENT) / 5 / 0.01
                                          / 1e12)


def test_atomic_roof_of_the_electron_pass(monkeypatch):
    # 10 launches of 2 ms, 1e8 steps; 0.6 additions per step against 2e10 additions/s
    stored = {"k_electron_pass": 50.0, "k_electron_pass_atomics": 0.6}
    monkeypatch.setattr(bench, "measured_traffic", lambda k: stored.get(k))
    acc = _acc(0.005, 0.020, 10, 10, 2e8, 1e8)
    assert "atomics" not in bench.roofline(acc, "water")        # no roof measured in this run
    acc.atomic_roof = 2e10
    r = bench.roofline(acc, "water")
    assert r["traffic"] == pytest.approx(50.0 * 1e7)
    assert r["atomics"]["achieved"] == pytest.approx(0.6 * 1e7 / 2e-3)
    assert r["atomics"]["frac"] == pytest.approx(0.6 * 1e7 / 2e-3 / 2e10)
    assert "atomics" not in bench.roofline(acc, "beamlets")     # counted on the water workload only


def test_traffic_is_dropped_when_the_sources_change(monkeypatch):
    monkeypatch.setitem(bench.TRAFFIC, "sources_sha256", "0" * 64)
    assert bench.measured_traffic("k_electron_pass") is None
