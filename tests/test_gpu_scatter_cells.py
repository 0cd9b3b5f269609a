"""GPU parity of the cell-list density scatter (owner-computes tiles with a
drift halo and a global-atomic fixup for strays) against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import counts_np, dev, host  # noqa: E402
from paper_1310_2041_amd import engine, hpf  # noqa: E402
from synth import workloads as wl  # noqa: E402


def cells_counts(st, R=None):
    if R is not None:
        st.R.copy_(dev(R, torch.float32))
    hpf.hpf_density_scatter_cells(st.R, st.T, st.mesh, st.K, st.cell_start, st.B, st.halo,
                                  st.counts, st.scatter_work)
    return counts_np(st.counts, st.K, tuple(st.mesh.M))


def drifted(R, L, sigma_cells, h_cell, seed):
    rng = np.random.default_rng(seed)
    out = R.copy()
    xyz = R[:, :3].astype(np.float64) + rng.standard_normal((len(R), 3)) * sigma_cells * h_cell
    Lf = np.broadcast_to(np.asarray(L, dtype=np.float32), (3,))
    out[:, :3] = np.mod(xyz, Lf.astype(np.float64)).astype(np.float32)
    out[:, :3] = np.where(out[:, :3] >= Lf, np.float32(0), out[:, :3])
    return out


CASES = [
    ("c1", lambda: wl.build(wl.SPECS["c1"]), 8, 1),
    ("noncubic_k3", lambda: wl.small_system(300, 12, (21.3, 17.9, 25.2), (20, 17, 24), K=3,
                                            n_solvent=4000, seed=61), 4, 2),
    ("halo0", lambda: wl.small_system(300, 12, 16.0, 15, seed=62), 8, 0),
    ("b3", lambda: wl.small_system(200, 10, 12.0, 11, seed=63), 3, 1),
]


@pytest.mark.parametrize("name,make,B,halo", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("sigma", [0.0, 0.4, 1.5, 6.0])
def test_cells_scatter_bit_exact_under_drift(name, make, B, halo, sigma):
    s0 = make()
    s, _ = wl.permuted(s0, seed=4)
    st = engine.HpfState.from_system(s, sort_brick=B, halo=halo)
    st.sort()
    R_sorted = host(st.R)
    T_sorted = host(st.T)
    h_cell = float(np.float32(s.L[0])) / st.mesh.M[0]
    R = drifted(R_sorted, s.L, sigma, h_cell, seed=int(sigma * 10) + B) if sigma else R_sorted
    st.counts.fill_(12345)                       # stale values must be overwritten
    got = cells_counts(st, R)
    want, sk = oracle.density(R, T_sorted, s.L, s.M, s.K)
    assert sk == 0
    assert np.array_equal(got, want)
    assert hpf.hpf_get_device_status() == 0


def test_cells_scatter_unbinnable_beads():
    s = wl.small_system(100, 10, 12.0, 12, seed=64)
    R = s.R.copy()
    R[5, 0] = np.nan                              # cannot be binned at sort time
    s.R[:] = R
    st = engine.HpfState.from_system(s)
    st.sort()
    R2 = host(st.R)
    R2[17, 1] = np.inf                            # becomes invalid after the sort
    R2[18, :3] = np.nan
    hpf.hpf_get_device_status(clear=True)
    got = cells_counts(st, R2)
    want, sk = oracle.density(R2, host(st.T), s.L, s.M, s.K)
    assert sk == 3
    assert np.array_equal(got, want)
    assert hpf.hpf_get_device_status() & hpf.HPF_FLAG_BAD_BEAD


def test_cells_scatter_rejects_small_mesh():
    s = wl.small_system(10, 10, 8.0, 9, seed=65)
    st = engine.HpfState.from_system(s, sort_brick=8, halo=1)
    st.sort()
    assert not st.cells_ok
    with pytest.raises(hpf.HpfError):
        hpf.hpf_density_scatter_cells(st.R, st.T, st.mesh, st.K, st.cell_start, 8, 1, st.counts,
                                      st.scatter_work)


@pytest.mark.slow
def test_cells_scatter_full_size_10m_after_dynamics():
    """10M-bead blend: counts after 10 steps of real dynamics past the sort."""
    s = wl.build(wl.SPECS["c3"])
    st = engine.HpfState.from_system(s)
    st.start(sort=True)
    st.run(9, sort_every=0)                       # beads drift away from the sort
    hpf.verlet_step(st.R, st.Vel, st.F, st.dt, st.box, 1)
    got = cells_counts(st)
    want, _ = oracle.density(host(st.R), host(st.T), s.L, s.M, s.K)
    assert np.array_equal(got, want)


def test_cells_scatter_eight_species_large_halo():
    """K = 8 with halo 2 needs more than 64 KiB of LDS per workgroup."""
    s = wl.small_system(400, 10, 20.0, 18, K=8, n_solvent=6000, seed=66)
    st = engine.HpfState.from_system(s, sort_brick=8, halo=2)
    st.sort()
    R = drifted(host(st.R), s.L, 0.8, 20.0 / 18, seed=3)
    got = cells_counts(st, R)
    want, _ = oracle.density(R, host(st.T), s.L, s.M, s.K)
    assert np.array_equal(got, want)
