"""Host-side checks of bench.py's reporting (no GPU): the kernel names it reads traffic for
must name the kernels the committed rocprofv3 summaries hold, the whole-step byte count
follows its formula, and a run asked for more than one GPU refuses."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1310_2041_amd.profile_summary import read_record  # noqa: E402

PROFILES = {
    "c3_ab_blend_10m": ["advance", "finish_potential", "field_gradient"],
    "c5_amphiphile_solvent_100m": ["advance", "finish_potential", "field_gradient"],
}


@pytest.mark.parametrize("workload", sorted(PROFILES))
def test_traffic_kernel_names_match_the_profiles(workload):
    rec = read_record(os.path.join(ROOT, "profiles", f"{workload}_step.md"))
    assert rec is not None
    names = list(rec["kernels"])
    for call in PROFILES[workload]:
        hits = [n for n in names if any(bench.rocprof_matches(p, n) for p in bench.ROCPROF_KERNELS[call])]
        assert hits, (call, names)
        for n in hits:
            assert rec["kernels"][n]["fetch_bytes"] is not None


def test_template_patterns_do_not_cross_kernels():
    assert bench.rocprof_matches("hpf::k_advance<", "hpf::k_advance<true, true, false, true>")
    assert not bench.rocprof_matches("hpf::k_advance<", "hpf::k_advance_scatter<true, 768, true, false, true>")
    assert bench.rocprof_matches("hpf::k_scatter_sum<true>", "hpf::k_scatter_sum<true>")
    assert not bench.rocprof_matches("hpf::k_scatter_sum<true>", "hpf::k_scatter_sum<false>")


def test_step_bytes_formula():
    r = {"N": 10_000_000, "K": 2, "nm": 128 ** 3}
    out = bench.step_bandwidth(r, 0.5)
    assert out["bytes_per_step"] == 70 * 10_000_000 + 32 * 2 * 128 ** 3
    assert out["achieved"] == pytest.approx(out["bytes_per_step"] / 0.5e-3 / 1e9, rel=1e-4)
    assert out["frac"] == pytest.approx(out["achieved"] / bench.HBM_PEAK_GBS, abs=1e-4)


def test_more_than_one_gpu_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode != 0
    assert "--gpus 1" in p.stderr
