"""GPU: hpf_density_scatter_cells_static (no workspace argument; a fixed device array
holds its stray list and partial boxes) gives the counts of hpf_density_scatter_cells bit
for bit, on two calls in a row, the second with a smaller input, so that what the first
call left in the array must not leak into the second. Both are checked against the FP64
oracle's counts as well. Called through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import counts_np, host  # noqa: E402
from paper_1310_2041_amd import engine, hpf  # noqa: E402
from synth import workloads as wl  # noqa: E402


def _sorted_state(s, B, halo, steps):
    """A system sorted by brick and then moved `steps` fused steps, so that some beads
    have left their brick's deposit box (they go through the stray list)."""
    st = engine.HpfState.from_system(s, sort_brick=B, halo=halo)
    st.start(sort=True)
    st.prime()
    if steps:
        st.run_fused(steps, report_every=0, sort_every=0)
    torch.cuda.synchronize()
    return st


def _both(st):
    ref = torch.zeros_like(st.counts)
    got = torch.full_like(st.counts, 12345)         # overwritten, need not be zero
    hpf.hpf_density_scatter_cells(st.R, st.T, st.mesh, st.K, st.cell_start, st.B, st.halo, ref,
                                  st.scatter_work)
    hpf.hpf_density_scatter_cells_static(st.R, st.T, st.mesh, st.K, st.cell_start, st.B, st.halo, got)
    torch.cuda.synchronize()
    return ref, got


def test_static_scratch_matches_workspace_call_twice():
    big = wl.build(wl.SPECS["c2"])                   # 1M beads, 64^3 mesh: 22 MB of scratch
    small = wl.small_system(300, 10, (13.7, 15.1, 14.2), (13, 15, 14), K=3, seed=5, n_solvent=700)
    hpf.hpf_get_device_status(clear=True)
    for s, B, halo, steps in ((big, 8, 2, 6), (small, 4, 1, 9)):
        st = _sorted_state(s, B, halo, steps)
        ref, got = _both(st)
        assert torch.equal(ref, got), (s.name, B, halo)
        R = host(st.R)
        T = host(st.T)
        want, _ = oracle.density(R, T, s.L, s.M, s.K)
        assert np.array_equal(counts_np(got, s.K, s.M), want)
        del st
    assert hpf.hpf_get_device_status() == 0
