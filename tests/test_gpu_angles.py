"""GPU: angle potentials (Bonded forces section) and the five-species lipid-like system.

angle_forces against the oracle's or_angles on the same FP32 positions (both
angle forms), the cell sort carrying the angle table, and whole force
evaluations and steps of the K = 5 lipid-in-water system against the oracle
(field, bond and angle forces compared separately)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import by_tag, dev, host, rel_max  # noqa: E402
from paper_1310_2041_amd import engine, hpf  # noqa: E402
from synth import workloads as wl  # noqa: E402


def lipids():
    return wl.lipid_system(2000, 96000)


def _oracle_angles(s, R=None):
    return oracle.angles(s.R if R is None else R, s.angles, s.angle_k, s.angle_theta0, s.angle_form,
                         s.L)


def test_angle_forces_match_oracle():
    s = lipids()
    R = dev(s.R, torch.float32)
    F = torch.zeros((s.N, 3), dtype=torch.float32, device="cuda")
    part = torch.zeros(hpf.HPF_NPART, dtype=torch.float64, device="cuda")
    hpf.angle_forces(R, dev(s.angles, torch.int32), s.angle_k, s.angle_theta0, s.angle_form, s.L, F,
                     e_part=part)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    hpf.hpf_reduce_partials(part, 1, out)
    Fo, Eo = _oracle_angles(s)
    err = rel_max(host(F)[:, :3], Fo)
    print(f"angle forces rel max-norm {err:.2e}; energy {host(out)[0]:.6e} vs {Eo:.6e}")
    assert err <= 1e-5
    assert host(out)[0] == pytest.approx(Eo, rel=1e-5)
    assert hpf.hpf_get_device_status() == 0


@pytest.mark.parametrize("form", [0, 1])
def test_single_angle_form_on_chains(form):
    """Every bead of 30,000 three-bead chains as middle or end, one angle type of each form."""
    rng = np.random.default_rng(4 + form)
    n_ch, L = 30000, 40.0
    start = rng.uniform(0, L, (n_ch, 3))
    d1 = rng.standard_normal((n_ch, 3))
    d2 = rng.standard_normal((n_ch, 3))
    pos = np.stack([start + 0.9 * d1 / np.linalg.norm(d1, axis=1, keepdims=True), start,
                    start + 1.1 * d2 / np.linalg.norm(d2, axis=1, keepdims=True)], 1).reshape(-1, 3)
    N = pos.shape[0]
    R = np.zeros((N, 3), np.float32)
    R[:, :3] = wl.wrap_f32(pos, L)
    tab = wl.angle_table([(3 * c, 3 * c + 1, 3 * c + 2, 0) for c in range(n_ch)], N)
    k, th0 = 7.5, 1.8
    F = torch.zeros((N, 3), dtype=torch.float32, device="cuda")
    hpf.angle_forces(dev(R, torch.float32), dev(tab, torch.int32), k, th0, form, (L, L, L), F)
    Fo, _ = oracle.angles(R, tab, k, th0, form, (L, L, L))
    err = rel_max(host(F)[:, :3], Fo)
    print(f"form {form}: rel max-norm {err:.2e}")
    assert err <= 1e-5


def test_sort_carries_the_angle_table():
    s, _ = wl.permuted(lipids(), seed=12)
    st = engine.HpfState.from_system(s)
    st.sort()
    perm, _ = oracle.sort_perm(s.R, s.tag, s.L, s.M, st.B)
    inv = np.empty(s.N, np.int64)
    inv[perm] = np.arange(s.N)
    a_old = s.angles[:, perm]
    idx_rows = (np.arange(a_old.shape[0]) % 3 != 2)[:, None]
    want = np.where(idx_rows, np.where(a_old >= 0, inv[np.maximum(a_old, 0)], -1), a_old)
    assert np.array_equal(host(st.angles), want)
    # the sorted table gives the same forces (by tag) as the input order
    st.F.zero_()
    st.angle_forces()
    F = by_tag(host(st.F)[:, :3], host(st.tag), s.N)
    Fo, _ = _oracle_angles(s)
    assert rel_max(F, by_tag(Fo, s.tag, s.N)) <= 1e-5
    assert hpf.hpf_get_device_status() == 0


def test_lipid_system_forces_match_oracle():
    """One force evaluation of the 120,000-bead K = 5 lipid system after the cell sort:
    counts bit-exact, field, bond and angle forces each within 1e-5 (relative max-norm),
    and the energies."""
    s = lipids()
    st = engine.HpfState.from_system(s)
    st.sort()
    hpf.hpf_density_scatter(st.R, st.T, st.mesh, st.K, st.counts)
    from gpu_util import counts_np
    c_or, sk = oracle.density(s.R, s.T, s.L, s.M, s.K)
    assert sk == 0 and np.array_equal(counts_np(st.counts, s.K, s.M), c_or)
    st.counts.zero_()
    tag = host(st.tag)
    st.field_forces(report=True)
    Ff = by_tag(host(st.F)[:, :3], tag, s.N)
    st.F.zero_()
    st.bond_forces(report=True)
    Fb = by_tag(host(st.F)[:, :3], tag, s.N)
    st.F.zero_()
    st.angle_forces(report=True)
    Fa = by_tag(host(st.F)[:, :3], tag, s.N)
    hpf.hpf_reduce_partials(st.part, engine.N_ROWS, st.energy)
    e = host(st.energy)
    Ff_or, Fb_or, e_or = oracle.forces(s)
    Fa_or, Ea_or = _oracle_angles(s)
    ef, eb, ea = rel_max(Ff, Ff_or), rel_max(Fb, Fb_or), rel_max(Fa, Fa_or)
    print(f"lipid K=5: field {ef:.2e}, bond {eb:.2e}, angle {ea:.2e}")
    assert ef <= 1e-5 and eb <= 1e-5 and ea <= 1e-5
    assert e[engine.ROW_W] == pytest.approx(e_or["W"], rel=1e-9)
    assert e[engine.ROW_EB] == pytest.approx(e_or["E_bond"], rel=1e-6)
    assert e[engine.ROW_EA] == pytest.approx(Ea_or, rel=1e-5)
    assert hpf.hpf_get_device_status() == 0


def test_lipid_steps_follow_oracle():
    """Ten steps of the lipid system (six calls with angles, a sort every 5 steps): per-step
    energies within 1e-4 of the oracle stepped by hand with the same pieces."""
    s = lipids()
    st = engine.HpfState.from_system(s)
    st.start(sort=True)
    trace = st.run(10, report_every=1, sort_every=5)
    Eg = np.array([[e["KE"], e["E_bond"], e["W"], e["E_angle"]] for e in trace])

    def force(R):
        Ff, Fb, e = oracle.forces(s, R=R)
        Fa, Ea = _oracle_angles(s, R)
        return Ff + Fb + Fa, e["W"], e["E_bond"], Ea

    R = s.R[:, :3].astype(np.float64)
    V = s.V[:, :3].astype(np.float64)
    F = force(R)[0]
    Eo = []
    for _ in range(10):
        R, V = oracle.verlet_half1(R, V, F, s.dt, s.L)
        F, W, Eb, Ea = force(R)
        V, out = oracle.verlet_half2(V, F, s.dt)
        Eo.append([out[0], Eb, W, Ea])
    Eo = np.asarray(Eo)
    rel = np.abs(Eg - Eo) / np.abs(Eo)
    print("max rel diff (KE, Eb, W, Eangle):", rel.max(0))
    assert rel.max() <= 1e-4
    assert hpf.hpf_get_device_status() == 0
    with pytest.raises(ValueError):
        st.step_fused()
