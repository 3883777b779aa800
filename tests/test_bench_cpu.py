"""CPU checks of bench.py's oracle leg: the serial full-step form, the
sampled form and its every-core variant all run, periodic and with the open
x boundary, on a small named workload.  The timed GPU legs need a GPU and run
only in bench.py itself."""
import pytest

import bench
import picgen


@pytest.mark.parametrize("xbc", [0, 1])
def test_cpu_baseline_sampled_and_all_cores(xbc):
    wl = picgen.WORKLOADS["2d3v_32x32_fp64"]
    r = bench.cpu_baseline(wl, full_limit=0, sample_n=256, xbc=xbc)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["value"] > 0
    assert r["all_cores"]["value"] > 0


@pytest.mark.parametrize("xbc", [0, 1])
def test_cpu_baseline_whole_steps(xbc):
    wl = picgen.WORKLOADS["2d3v_32x32_fp64"]
    r = bench.cpu_baseline(wl, min_seconds=0.05, max_steps=2, xbc=xbc)
    assert r["kind"] == "oracle" and r["value"] > 0
