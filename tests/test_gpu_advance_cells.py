"""GPU: the brick-box fused pass (hpf_advance_cells) against hpf_advance.

Both compute the same per-bead arithmetic; only where the gradient corners are
read from differs (a brick's LDS box or memory), so every bead state and force
must agree bit for bit, for beads inside their brick box, beads that drifted
out of it, and beads the sort could not bin. The energy partials are grouped
differently, so the reduced energies agree to FP64 rounding only.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import dev, host  # noqa: E402
from paper_1310_2041_amd import engine, hpf  # noqa: E402
from synth import workloads as wl  # noqa: E402


def drifted(R, L, sigma_cells, h_cell, seed):
    rng = np.random.default_rng(seed)
    out = R.copy()
    xyz = R[:, :3].astype(np.float64) + rng.standard_normal((len(R), 3)) * sigma_cells * h_cell
    Lf = np.broadcast_to(np.asarray(L, dtype=np.float32), (3,))
    out[:, :3] = np.mod(xyz, Lf.astype(np.float64)).astype(np.float32)
    out[:, :3] = np.where(out[:, :3] >= Lf, np.float32(0), out[:, :3])
    return out


def field_of(st):
    """Counts (any-order scatter), potential and gradient of the current positions."""
    hpf.hpf_density_scatter(st.R, st.T, st.mesh, st.K, st.counts)
    hpf.hpf_field_potential(st.counts, st.mesh, st.field, st.V, None)
    hpf.hpf_field_gradient(st.V, st.mesh, st.K, st.G)


def both(st, halo, inv_mass=None):
    bonds = st.bonds if st.bonds.shape[0] else None
    out = []
    for cells in (False, True):
        Rn = torch.empty_like(st.R)
        Vel = st.Vel.clone()
        F = torch.empty_like(st.R)
        part = torch.zeros((5, hpf.HPF_NPART), dtype=torch.float64, device="cuda")
        e = torch.zeros(5, dtype=torch.float64, device="cuda")
        kw = dict(inv_mass=inv_mass, F_out=F, e_part=part[0], kin_part=part[1:5])
        if cells:
            hpf.hpf_advance_cells(st.R, Rn, Vel, st.T, st.mesh, st.K, st.G, bonds, st.k_bond, st.r0,
                                  st.box, st.dt, st.cell_start, st.B, halo, **kw)
        else:
            hpf.hpf_advance(st.R, Rn, Vel, st.T, st.mesh, st.K, st.G, bonds, st.k_bond, st.r0,
                            st.box, st.dt, **kw)
        hpf.hpf_reduce_partials(part, 5, e)
        out.append((host(Rn), host(Vel), host(F), host(e)))
    return out


def assert_same(a, b):
    for x, y, name in zip(a[:3], b[:3], ("R_next", "Vel", "F")):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), name
    np.testing.assert_allclose(b[3], a[3], rtol=1e-12, atol=1e-9)


CASES = [
    ("c1", lambda: wl.build(wl.SPECS["c1"]), 8),
    ("noncubic_k3", lambda: wl.small_system(300, 12, (21.3, 17.9, 25.2), (20, 17, 24), K=3,
                                            n_solvent=4000, seed=61), 4),
    ("b3_small_mesh", lambda: wl.small_system(200, 10, 12.0, 11, seed=63), 3),
    ("ragged_bricks", lambda: wl.small_system(137, 7, (19.7, 14.3, 9.1), (19, 13, 9), seed=65), 8),
]


@pytest.mark.parametrize("name,make,B", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("halo", [0, 1, 2])
@pytest.mark.parametrize("sigma", [0.0, 0.6, 3.0])
def test_advance_cells_bitwise_under_drift(name, make, B, halo, sigma):
    if halo >= B:
        pytest.skip("halo must be below the brick edge")
    s, _ = wl.permuted(make(), seed=3)
    st = engine.HpfState.from_system(s, sort_brick=B)
    st.sort()
    if sigma:
        h_cell = float(np.float32(s.L[0] if np.ndim(s.L) == 0 else s.L[0])) / st.mesh.M[0]
        st.R.copy_(dev(drifted(host(st.R), s.L, sigma, h_cell, seed=int(10 * sigma) + B), torch.float32))
    field_of(st)
    a, b = both(st, halo)
    assert_same(a, b)
    assert hpf.hpf_get_device_status() == 0


def test_advance_cells_bond_length_and_masses():
    s = wl.small_system(250, 10, 16.0, 16, seed=66)
    s.r0 = 0.75
    st = engine.HpfState.from_system(s)
    st.sort()
    field_of(st)
    rng = np.random.default_rng(8)
    im = dev(rng.uniform(0.5, 2.0, st.N).astype(np.float32), torch.float32)
    a, b = both(st, 1, inv_mass=im)
    assert_same(a, b)
    assert hpf.hpf_get_device_status() == 0


def test_advance_cells_unbinnable_beads():
    s = wl.small_system(100, 10, 12.0, 12, seed=64)
    s.R[5, 0] = np.nan                             # cannot be binned at sort time
    st = engine.HpfState.from_system(s)
    st.sort()
    R = host(st.R)
    R[17, 1] = np.inf                              # invalid after the sort
    st.R.copy_(dev(R, torch.float32))
    field_of(st)
    hpf.hpf_get_device_status(clear=True)
    a, b = both(st, 1)
    for x, y, name in zip(a[:3], b[:3], ("R_next", "Vel", "F")):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), name
    assert hpf.hpf_get_device_status(clear=True) & hpf.HPF_FLAG_BAD_BEAD


def test_advance_cells_lds_limit():
    s = wl.small_system(50, 10, 12.0, 12, K=8, seed=67)
    st = engine.HpfState.from_system(s)
    st.sort()
    field_of(st)
    assert not hpf.advance_cells_fits(8, 8, 1) and hpf.advance_cells_fits(8, 8, 0)
    with pytest.raises(hpf.HpfError):
        hpf.hpf_advance_cells(st.R, torch.empty_like(st.R), st.Vel.clone(), st.T, st.mesh, 8, st.G,
                              st.bonds, st.k_bond, st.r0, st.box, st.dt, st.cell_start, 8, 1)
    a, b = both(st, 0)
    assert_same(a, b)


def test_engine_cells_advance_matches_plain_over_steps():
    s = wl.build(wl.SPECS["c2"])
    a = engine.HpfState.from_system(s, advance="plain")
    b = engine.HpfState.from_system(s, advance="cells")
    for st in (a, b):
        st.start(sort=True)
        st.prime()
    ea = a.run_fused(25, report_every=25, sort_every=10)
    eb = b.run_fused(25, report_every=25, sort_every=10)
    assert b.uses_cells_advance() and not a.uses_cells_advance()
    for x, y in zip(a.host_beads(), b.host_beads()):
        assert np.array_equal(x, y)
    for key in ("KE", "E_bond", "W", "E_tot"):
        assert eb[-1][key] == pytest.approx(ea[-1][key], rel=1e-12)
    assert hpf.hpf_get_device_status() == 0


def test_plain_pass_bond_table_widths():
    """hpf_advance: a three-row bond table (third row all -1) takes the general bead loop and
    must move beads exactly as the two-row table does (the software-pipelined loop); with no
    table at all it must equal a table of -1 only."""
    s = wl.build(wl.SPECS["c1"])
    st = engine.HpfState.from_system(s)
    st.sort()
    field_of(st)
    pad = torch.full((1, st.N), -1, dtype=torch.int32, device="cuda")

    def run(bonds):
        Rn, Vel = torch.empty_like(st.R), st.Vel.clone()
        hpf.hpf_advance(st.R, Rn, Vel, st.T, st.mesh, st.K, st.G, bonds, st.k_bond, st.r0, st.box, st.dt)
        return host(Rn), host(Vel)

    two = run(st.bonds)
    three = run(torch.cat([st.bonds, pad]).contiguous())
    for x, y in zip(two, three):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    none = run(None)
    empty = run(torch.full((2, st.N), -1, dtype=torch.int32, device="cuda"))
    for x, y in zip(none, empty):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    assert hpf.hpf_get_device_status() == 0
