"""Host-side logic of the benchmark (no GPU): the one-GPU refusal, the roofline arithmetic and
the tie between the committed hardware-counter summaries and the trace kernel's sources."""
import glob
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (imports nothing that touches a GPU at module level)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


class _CountedWork:
    """Stands in for the binding: the counted work per unit that the library exports."""
    @staticmethod
    def work_per_unit():
        return {"step_flops": 474.0, "sample_flops": 151.0, "freq_flops": 23.0}


@pytest.mark.parametrize("fp64_transfer,n_nu", [(False, 1), (True, 4)])
def test_roofline_is_counted_work_over_kernel_time(fp64_transfer, n_nu):
    st = {"ray_steps": 920_000_000, "samples": 382_000_000}
    ms = 25.0
    r = bench.roofline_of(_CountedWork, st, ms, fp64_transfer, n_nu)
    flops = 920e6 * 474 + 382e6 * 151 + (382e6 * n_nu * 23 if fp64_transfer else 0)
    assert r["achieved"] == pytest.approx(flops / 25e-3 / 1e12, rel=1e-12)
    assert r["peak"] == 78.6 and r["unit"] == "TFLOP/s" and r["bound"] == "alu"
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6, rel=1e-12)
    assert r["traffic"] is None


def test_counter_summaries_belong_to_the_current_trace_kernel():
    """Every committed summary that names a trace-kernel build names the one the sources build,
    and the HBM traffic the benchmark reports comes from that build's counters (the benchmark
    reports null traffic otherwise)."""
    from paper_1801_10452_amd import raptor as R
    build = R.kernel_build_id()
    with open(os.path.join(ROOT, "profiles", "trace_kernel_traffic.json")) as f:
        tj = json.load(f)
    assert tj["kernel_build"] == build
    assert tj["bytes_per_launch"] > 0 and tj["fetch_factor"] > 0 and tj["write_factor"] > 0
    named = {}
    for p in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        with open(p) as f:
            ids = set(re.findall(r"[Kk]ernel build `?([0-9a-f]{16})", f.read()))
        if ids:
            named[os.path.basename(p)] = ids
    assert named, "no summary names its kernel build"
    stale = {k: v for k, v in named.items() if v != {build}}
    assert not stale, f"summaries of another build than {build}: {stale}"
