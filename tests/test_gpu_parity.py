"""GPU parity of every C-ABI entry point against the FP64 oracle.

Each test calls the HIP library through its binding on seeded synthetic
inputs and compares element by element with the oracle on the same inputs:
integer work (counts, sort permutation, renumbered bonds) bit-exactly,
floating point within the stated tolerance.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import by_tag, counts_np, dev, host, rel_max  # noqa: E402
from paper_1310_2041_amd import engine, hpf  # noqa: E402
from synth import workloads as wl  # noqa: E402

I64 = torch.int64


def _pos3(xyz):
    return np.ascontiguousarray(np.asarray(xyz, dtype=np.float32).reshape(-1, 3))


def gpu_counts(R, T, L, M, K):
    mesh = hpf.hpf_mesh_make(L, M, len(T))
    nm = mesh.M[0] * mesh.M[1] * mesh.M[2]
    c = torch.zeros((K, nm), dtype=I64, device="cuda")
    hpf.hpf_density_scatter(dev(R, torch.float32), dev(T, torch.uint8), mesh, K, c)
    return counts_np(c, K, tuple(mesh.M))


def _systems():
    yield "c1", wl.build(wl.SPECS["c1"])
    yield "ragged_noncubic_k3", wl.small_system(97, 13, (11.3, 7.9, 15.2), (11, 8, 17), K=3,
                                                n_solvent=1001, seed=12)
    yield "tiny_mesh", wl.small_system(5, 4, 3.1, 3, seed=13)
    yield "k8", wl.small_system(40, 8, 9.0, 9, K=8, n_solvent=700, seed=14)


# ---------------------------------------------------------------- scatter --

@pytest.mark.parametrize("name,s", list(_systems()), ids=lambda x: x if isinstance(x, str) else "")
def test_scatter_counts_bit_exact(name, s):
    c_or, sk = oracle.density(s.R, s.T, s.L, s.M, s.K)
    assert sk == 0
    assert np.array_equal(gpu_counts(s.R, s.T, s.L, s.M, s.K), c_or)
    sp, _ = wl.permuted(s)             # storage order must not matter
    assert np.array_equal(gpu_counts(sp.R, sp.T, sp.L, sp.M, sp.K), c_or)
    assert hpf.hpf_get_device_status() == 0


@pytest.mark.parametrize("n", [0, 1, 2, 63, 2047, 2048, 2049, 5000])
def test_scatter_ragged_sizes(n):
    rng = np.random.default_rng(n)
    L, M = (6.7, 5.3, 9.1), (7, 5, 10)
    R = _pos3(rng.random((n, 3)) * np.array(L))
    T = rng.integers(0, 2, n).astype(np.uint8)
    c_or, _ = oracle.density(R, T, L, M, 2)
    assert np.array_equal(gpu_counts(R, T, L, M, 2), c_or)


def test_scatter_edge_positions_and_bad_beads():
    L, M = 8.0, 8
    Lf = np.float32(L)
    xs = [0.0, np.nextafter(Lf, np.float32(0)), -1e-7, -0.3, 7.999, 8.0, 11.5, -9.25, 1e-38]
    R = _pos3([[x, y, z] for x in xs for y in xs[:4] for z in xs[4:]])
    T = (np.arange(len(R)) % 2).astype(np.uint8)
    c_or, sk = oracle.density(R, T, L, M, 2)
    assert sk == 0
    hpf.hpf_get_device_status(clear=True)
    assert np.array_equal(gpu_counts(R, T, L, M, 2), c_or)
    assert hpf.hpf_get_device_status() == 0
    bad = _pos3([[1.0, 1.0, 1.0], [np.nan, 1, 1], [1, np.inf, 1], [1e30, 1, 1], [2, 2, 2]])
    Tb = np.array([0, 0, 0, 0, 7], np.uint8)
    c_or, sk = oracle.density(bad, Tb, L, M, 2)
    assert sk == 4
    assert np.array_equal(gpu_counts(bad, Tb, L, M, 2), c_or)
    assert hpf.hpf_get_device_status() & hpf.HPF_FLAG_BAD_BEAD


def test_scatter_spread_chunk_falls_back_exactly():
    """Beads scattered over the whole box (no locality) take the global-atomic path."""
    rng = np.random.default_rng(5)
    L, M = 64.0, 64
    R = _pos3(rng.random((50000, 3)) * L)
    T = rng.integers(0, 3, 50000).astype(np.uint8)
    c_or, _ = oracle.density(R, T, L, M, 3)
    assert np.array_equal(gpu_counts(R, T, L, M, 3), c_or)


# -------------------------------------------------------------- potential --

@pytest.mark.parametrize("name,s", list(_systems()), ids=lambda x: x if isinstance(x, str) else "")
def test_potential_matches_oracle_and_clears_counts(name, s):
    c_or, _ = oracle.density(s.R, s.T, s.L, s.M, s.K)
    V_or, W_or = oracle.potential(c_or, s.L, s.M, s.N, s.kT, s.inv_kappa, s.chi)
    mesh = hpf.hpf_mesh_make(s.L, s.M, s.N)
    field = hpf.make_field(s.K, s.kT, s.inv_kappa, s.chi)
    nm = int(np.prod(s.M))
    counts = dev(c_or.reshape(s.K, nm).view(np.int64), I64)
    V = torch.empty((s.K, nm), dtype=torch.float32, device="cuda")
    part = torch.zeros(hpf.HPF_NPART, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    hpf.hpf_field_potential(counts, mesh, field, V, part)
    hpf.hpf_reduce_partials(part, 1, out)
    Vg = host(V).reshape(V_or.shape)
    assert np.all(np.abs(Vg - V_or) <= 2.0 ** -23 * np.abs(V_or) + 1e-30)
    assert float(host(out)[0]) == pytest.approx(W_or, rel=1e-12)
    assert not host(counts).any()


def test_potential_overflow_flag():
    L, M = 6.0, 6
    c = np.zeros((1, 6, 6, 6), np.uint64)
    c[0, 1, 2, 3] = np.uint64(1) << np.uint64(62)
    mesh = hpf.hpf_mesh_make(L, M, 10)
    field = hpf.make_field(1, 1.0, 10.0, [[0.0]])
    V = torch.empty((1, 216), dtype=torch.float32, device="cuda")
    hpf.hpf_get_device_status(clear=True)
    hpf.hpf_field_potential(dev(c.reshape(1, -1).view(np.int64), I64), mesh, field, V)
    assert hpf.hpf_get_device_status() & hpf.HPF_FLAG_OVERFLOW


# --------------------------------------------------------------- gradient --

@pytest.mark.parametrize("L,M,K", [(18.8, (20, 20, 20), 2), ((11.3, 7.9, 15.2), (11, 8, 17), 3),
                                   (3.1, (3, 3, 3), 1), (69.3, (64, 64, 64), 2),
                                   ((40.0, 9.0, 5.0), (130, 9, 5), 2)])
def test_gradient_matches_oracle(L, M, K):
    rng = np.random.default_rng(sum(M))
    V = (rng.standard_normal((K, M[2], M[1], M[0])) * 3.0).astype(np.float32)
    G_or = oracle.gradient(V.astype(np.float64), L, M)
    mesh = hpf.hpf_mesh_make(L, M, 1000)
    nm = int(np.prod(M))
    G = torch.empty((K, nm, 3), dtype=torch.float32, device="cuda")
    hpf.hpf_field_gradient(dev(V.reshape(K, nm), torch.float32), mesh, K, G)
    Gg = host(G).reshape(K, M[2], M[1], M[0], 3)
    assert rel_max(Gg, G_or) <= 1e-6
    assert np.all(np.abs(Gg - G_or) <= 4e-7 * np.abs(G_or) + 1e-6 * np.abs(G_or).max())


# ----------------------------------------------------------------- gather --

@pytest.mark.parametrize("name,s", list(_systems()), ids=lambda x: x if isinstance(x, str) else "")
def test_gather_matches_oracle(name, s):
    rng = np.random.default_rng(3)
    nm = int(np.prod(s.M))
    G = rng.standard_normal((s.K, nm, 3)).astype(np.float32)
    F_or = oracle.gather(s.R, s.T, s.L, s.M, G.reshape(s.K, *s.M[::-1], 3).astype(np.float64))
    mesh = hpf.hpf_mesh_make(s.L, s.M, s.N)
    F = torch.full((s.N, 3), 7.0, dtype=torch.float32, device="cuda")
    hpf.hpf_force_gather(dev(s.R, torch.float32), dev(s.T, torch.uint8), mesh, s.K,
                         dev(G, torch.float32), F)
    Fg = host(F)
    assert rel_max(Fg[:, :3], F_or) <= 1e-6


# ------------------------------------------------------------------ bonds --

@pytest.mark.parametrize("r0", [0.0, 0.45])
def test_bonds_match_oracle(r0):
    s = wl.small_system(300, 20, 9.7, 9, seed=21)
    F_or, E_or = oracle.bonds(s.R, s.bonds, s.k_bond, r0, s.L)
    F0 = np.random.default_rng(1).standard_normal((s.N, 3)).astype(np.float32)
    F = dev(F0, torch.float32)
    part = torch.zeros(hpf.HPF_NPART, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    hpf.bond_forces(dev(s.R, torch.float32), dev(s.bonds, torch.int32), s.k_bond, r0, s.L, F, part)
    hpf.hpf_reduce_partials(part, 1, out)
    Fg = host(F)
    assert rel_max(Fg[:, :3] - F0[:, :3], F_or) <= 2e-6
    assert float(host(out)[0]) == pytest.approx(E_or, rel=1e-6)


def test_bonds_across_the_seam_of_a_large_box():
    """Bonds that straddle the periodic boundary of the 322-edge box keep full precision."""
    L = 322.0
    rng = np.random.default_rng(4)
    n = 2000
    xi = rng.random((n, 3)) * 0.8
    xj = np.mod(xi - 0.3 - rng.random((n, 3)) * 0.6, L)
    R = _pos3(np.concatenate([xi, xj]))
    bonds = np.full((1, 2 * n), -1, np.int32)
    bonds[0, :n] = np.arange(n, 2 * n)
    bonds[0, n:] = np.arange(n)
    F_or, _ = oracle.bonds(R, bonds, 100.0, 0.0, L)
    F = torch.zeros((2 * n, 3), dtype=torch.float32, device="cuda")
    hpf.bond_forces(dev(R, torch.float32), dev(bonds, torch.int32), 100.0, 0.0, L, F)
    assert rel_max(host(F)[:, :3], F_or) <= 1e-6


# ----------------------------------------------------------------- verlet --

def test_verlet_halves_match_oracle():
    s = wl.small_system(100, 10, 7.0, 7, seed=31)
    rng = np.random.default_rng(2)
    F0 = (rng.standard_normal((s.N, 3)) * 50).astype(np.float32)
    R1o, V1o = oracle.verlet_half1(s.R, s.V, F0[:, :3], 0.03, s.L)
    R, Vel, F = dev(s.R, torch.float32), dev(s.V, torch.float32), dev(F0, torch.float32)
    hpf.verlet_step(R, Vel, F, 0.03, s.L, 1)
    dR = host(R)[:, :3] - R1o
    dR -= np.float32(7.0) * np.rint(dR / np.float32(7.0))
    assert np.abs(dR).max() <= 4e-6
    assert rel_max(host(Vel)[:, :3], V1o) <= 1e-6
    Rh = host(R)[:, :3]
    assert np.all((Rh >= 0) & (Rh < np.float32(7.0)))
    V2o, out = oracle.verlet_half2(host(Vel)[:, :3], F0[:, :3], 0.03)
    part = torch.zeros((4, hpf.HPF_NPART), dtype=torch.float64, device="cuda")
    e = torch.zeros(4, dtype=torch.float64, device="cuda")
    hpf.verlet_step(None, Vel, F, 0.03, s.L, 2, kin_part=part)
    hpf.hpf_reduce_partials(part, 4, e)
    assert rel_max(host(Vel)[:, :3], V2o) <= 1e-6
    assert host(e)[0] == pytest.approx(out[0], rel=1e-6)
    assert np.allclose(host(e)[1:], out[1:], atol=1e-4 * np.sqrt(s.N))


def test_verlet_nonfinite_flag():
    R = dev(_pos3([[1.0, 1.0, 1.0]]), torch.float32)
    Vel = dev(_pos3([[np.inf, 0.0, 0.0]]), torch.float32)
    F = torch.zeros((1, 3), dtype=torch.float32, device="cuda")
    hpf.hpf_get_device_status(clear=True)
    hpf.verlet_step(R, Vel, F, 0.03, 5.0, 1)
    assert hpf.hpf_get_device_status() & hpf.HPF_FLAG_NONFINITE


# ------------------------------------------------------------------- sort --

@pytest.mark.parametrize("B", [8, 4, 3])
def test_sort_matches_oracle_permutation(B):
    s0 = wl.small_system(400, 10, (13.1, 9.7, 21.0), (13, 10, 21), seed=41)
    s, _ = wl.permuted(s0)
    perm, keys = oracle.sort_perm(s.R, s.tag, s.L, s.M, B)
    st = engine.HpfState.from_system(s, sort_brick=B)
    st.sort()
    R, Vel, T, tag, bonds = st.host_beads()
    assert np.array_equal(tag, s.tag[perm])
    assert np.array_equal(R, s.R[perm])
    assert np.array_equal(Vel, s.V[perm])
    assert np.array_equal(T, s.T[perm])
    inv = np.empty(s.N, np.int64)
    inv[perm] = np.arange(s.N)
    b_old = s.bonds[:, perm]
    assert np.array_equal(bonds, np.where(b_old >= 0, inv[np.maximum(b_old, 0)], -1))
    nk = hpf.sort_key_count(st.mesh, B)
    cs = host(st.cell_start)
    expect = np.searchsorted(np.sort(keys), np.arange(nk + 2), side="left")
    expect[nk + 1] = s.N
    assert np.array_equal(cs, expect)
    assert hpf.hpf_get_device_status() == 0


@pytest.mark.parametrize("n_chains", [800, 1500])
def test_sort_single_dense_brick(n_chains):
    """All beads in one brick (8000 and 15000 beads): still the oracle's order, no flag."""
    s0 = wl.small_system(n_chains, 10, 7.0, 7, seed=43)
    s, _ = wl.permuted(s0, seed=2)
    st = engine.HpfState.from_system(s, sort_brick=8)
    hpf.hpf_get_device_status(clear=True)
    st.sort()
    R, Vel, T, tag, bonds = st.host_beads()
    perm, _ = oracle.sort_perm(s.R, s.tag, s.L, s.M, 8)
    assert np.array_equal(tag, s.tag[perm])
    assert np.array_equal(R, s.R[perm])
    assert hpf.hpf_get_device_status(clear=True) == 0


@pytest.mark.parametrize("fault", ["repeated", "out_of_range"])
def test_sort_rejects_bad_tags_safely(fault):
    """Tags that are not a permutation of [0, N) raise the flag; every index the sort writes
    stays inside [0, N)."""
    s = wl.small_system(200, 10, 12.0, 12, seed=44)
    if fault == "repeated":
        s.tag[7] = s.tag[8]
    else:
        s.tag[7] = s.N + 5
    st = engine.HpfState.from_system(s)
    hpf.hpf_get_device_status(clear=True)
    st.sort()
    flags = hpf.hpf_get_device_status(clear=True)
    assert flags & hpf.HPF_FLAG_SORT_ORDER
    R, Vel, T, tag, bonds = st.host_beads()
    assert np.isin(R[:, 0], s.R[:, 0]).all()                   # gathered from real input rows
    assert ((bonds >= -1) & (bonds < s.N)).all()


def test_sort_is_canonical_for_any_input_order():
    s = wl.build(wl.SPECS["c1"])
    sp, _ = wl.permuted(s, seed=5)
    a = engine.HpfState.from_system(s)
    b = engine.HpfState.from_system(sp)
    a.sort()
    b.sort()
    for x, y in zip(a.host_beads(), b.host_beads()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("n_chains,chain_len", [(1, 1), (1, 3), (7, 5), (300, 7), (1100, 20)])
def test_per_bead_kernels_ragged_sizes(n_chains, chain_len):
    """Tiny and ragged bead counts through gather, bonds, Verlet and the fused pass."""
    s = wl.small_system(n_chains, chain_len, 9.0, 9, seed=n_chains + chain_len)
    rng = np.random.default_rng(1)
    nm = 9 ** 3
    G = rng.standard_normal((2, nm, 3)).astype(np.float32)
    F_or = oracle.gather(s.R, s.T, s.L, s.M, G.reshape(2, 9, 9, 9, 3).astype(np.float64))
    Fb_or, _ = oracle.bonds(s.R, s.bonds, s.k_bond, s.r0, s.L)
    mesh = hpf.hpf_mesh_make(s.L, s.M, s.N)
    R, T, Gd = dev(s.R, torch.float32), dev(s.T, torch.uint8), dev(G, torch.float32)
    bonds = dev(s.bonds, torch.int32)
    F = torch.zeros((s.N, 3), dtype=torch.float32, device="cuda")
    hpf.hpf_force_gather(R, T, mesh, 2, Gd, F)
    assert rel_max(host(F)[:, :3], F_or) <= 1e-6
    hpf.bond_forces(R, bonds, s.k_bond, s.r0, s.L, F)
    assert rel_max(host(F)[:, :3], F_or + Fb_or) <= 1e-6
    # fused pass == separate calls, bit for bit
    V1 = dev(s.V, torch.float32)
    V2 = V1.clone()
    R1 = R.clone()
    part1 = torch.zeros((4, hpf.HPF_NPART), dtype=torch.float64, device="cuda")
    part2 = torch.ones((4, hpf.HPF_NPART), dtype=torch.float64, device="cuda")   # stale slots
    hpf.verlet_step(None, V1, F, 0.03, s.L, 2, kin_part=part1)
    hpf.verlet_step(R1, V1, F, 0.03, s.L, 1)
    R2 = torch.empty_like(R)
    hpf.hpf_advance(R, R2, V2, T, mesh, 2, Gd, bonds, s.k_bond, s.r0, s.L, 0.03, kin_part=part2)
    assert torch.equal(R1, R2) and torch.equal(V1, V2)
    o1 = torch.zeros(4, dtype=torch.float64, device="cuda")
    o2 = torch.zeros(4, dtype=torch.float64, device="cuda")
    hpf.hpf_reduce_partials(part1, 4, o1)
    hpf.hpf_reduce_partials(part2, 4, o2)
    # the fused pass groups its partials by 512-bead chunks, the separate call by 256
    np.testing.assert_allclose(host(o2), host(o1), rtol=1e-12, atol=1e-9)
