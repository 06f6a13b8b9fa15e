"""The benchmark's byte accounting and roofline arithmetic (CPU only): the algorithmic
bytes per unit of the store-all scheme and of the fused LB step, worked by hand for the
benchmark workloads, and the roofline fields computed from a given launch time."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bytes_per_update(bench):
    # s (stored G_s written and read once) + nsp (s + 8) / (2 N): one field factor per species
    # read and one FP64 density per species written per evaluation of 2 N updates
    melt32 = bench.make_workloads("melt64_a8b8", "fp32")[0]           # N 16, 2 species
    ves32 = bench.make_workloads("vesicle128_a3b9s", "fp32")[0]      # N 12, 3 species
    melt64 = bench.make_workloads("melt64_a8b8", "fp64")[0]
    assert bench.bytes_per_update(melt32) == 4 + 2 * 12 / 32 == 4.75
    assert bench.bytes_per_update(ves32) == 4 + 3 * 12 / 24 == 5.5
    assert bench.bytes_per_update(melt64) == 8 + 2 * 16 / 32 == 9.0


def test_lb_bytes_per_site(bench):
    # 19 populations read and written, force read, density and velocity written
    assert bench.lb_bytes_per_site(bench.make_workloads("vesicle128_a3b9s", "fp32")[0]) == 4 * 45 == 180
    assert bench.lb_bytes_per_site(bench.make_workloads("melt64_a8b8", "fp64")[0]) == 8 * 45 == 360


def test_rooflines_from_launch_times(bench):
    wls = bench.make_workloads("vesicle128_a3b9s", "fp32")
    V = 128 ** 3
    # 1 000 paired launches of 19.5 us and 10 LB steps of 74 us
    timing = {"pair": (19.5, 1000), "bwd": (3.9, 100), "lb": (0.74, 10)}
    kernels, prop, lb = bench.rooflines(timing, wls, (32, 8, 4, -1), "vesicle128_a3b9s")
    assert kernels["pair"]["avg_us"] == pytest.approx(19.5)
    units = V * 23 / 12          # forward steps 1..12 and backward steps 12..2 in 12 launches
    assert prop["updates_per_launch"] == pytest.approx(units)
    assert prop["algorithmic_bytes_per_launch"] == pytest.approx(5.5 * units)
    achieved = 5.5 * units / 19.5e-6 / 1e9
    assert prop["achieved"] == pytest.approx(achieved) and prop["frac"] == pytest.approx(achieved / 8000.0)
    assert prop["traffic"] == 70.31e6
    assert prop["traffic_frac"] == pytest.approx(70.31e6 / 19.5e-6 / 1e9 / 8000.0)
    assert lb["mlups"] == pytest.approx(V / 74e-6 / 1e6)
    assert lb["frac"] == pytest.approx(180 * V / 74e-6 / 1e9 / 8000.0)
    assert lb["traffic"] == 436.68e6
    # counters taken for one tiling do not describe another
    _, prop2, _ = bench.rooflines({"pair": (19.5, 1000)}, wls, (32, 8, 2, -1), "vesicle128_a3b9s")
    assert prop2["traffic"] is None and prop2["traffic_frac"] is None
