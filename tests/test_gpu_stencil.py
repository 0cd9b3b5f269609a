"""GPU: the paper-literal staggered stencil (Algorithm 1 Kernels 3-4, read with the
nearest mesh point and the fraction ratios 1/2 -+ delta) against the oracle's
or_gather_staggered, on identical FP32 potentials, and whole steps of it."""
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

CASES = [
    ("c1", lambda: wl.build(wl.SPECS["c1"])),
    ("noncubic_k3", lambda: wl.small_system(300, 12, (21.3, 17.9, 25.2), (20, 17, 24), K=3,
                                            n_solvent=4000, seed=61)),
    ("ragged", lambda: wl.small_system(137, 7, (19.7, 14.3, 9.1), (19, 13, 9), seed=65)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_staggered_gather_matches_oracle(name, make):
    s = make()
    M = tuple(s.M)
    rng = np.random.default_rng(3)
    V = rng.standard_normal((s.K, M[2], M[1], M[0])).astype(np.float32)
    mesh = hpf.hpf_mesh_make(s.L, M, s.N)
    R, T = dev(s.R, torch.float32), dev(s.T, torch.uint8)
    F = torch.full((s.N, 3), 7.0, dtype=torch.float32, device="cuda")
    hpf.hpf_force_gather_staggered(R, T, mesh, s.K, dev(V.reshape(s.K, -1), torch.float32), F)
    want = oracle.gather_staggered(s.R, s.T, s.L, M, V.astype(np.float64), np.eye(s.K))
    err = rel_max(host(F)[:, :3], want)
    print(f"{name}: rel max-norm {err:.2e}")
    assert err <= 1e-6
    assert hpf.hpf_get_device_status() == 0


def test_staggered_forces_of_the_melt_match_the_paper_order():
    """Counts, potential and the staggered gather on the GPU against the oracle's paper-order
    force (differences of phi per species, then kT chi + 1/kappa) at full C1 size."""
    s = wl.build(wl.SPECS["c1"])
    st = engine.HpfState.from_system(s, stencil="staggered")
    st.sort()
    st.field_forces()
    F = by_tag(host(st.F)[:, :3].astype(np.float64), host(st.tag), s.N)
    counts, _ = oracle.density(s.R, s.T, s.L, s.M, s.K)
    vol = float(np.prod(np.asarray(s.L, dtype=np.float32).astype(np.float64)))
    nm = int(np.prod(s.M))
    phi = counts.astype(np.float64) / (2.0 ** 48 * (s.N / vol) * (vol / nm))
    A = s.kT * np.asarray(s.chi) + s.inv_kappa
    want = oracle.gather_staggered(s.R, s.T, s.L, s.M, phi, A)
    err = rel_max(F, want)
    print(f"c1 staggered field force: rel max-norm {err:.2e}")
    assert err <= 1e-5


def test_staggered_steps_follow_oracle():
    """Ten velocity-Verlet steps with the staggered field force: positions of every bead
    within 1e-5 of the box (relative), stepping the oracle's force by hand."""
    s = wl.build(wl.SPECS["c1"])
    st = engine.HpfState.from_system(s, stencil="staggered")
    st.start(sort=True)
    st.run(10, report_every=0, sort_every=5)
    A = s.kT * np.asarray(s.chi) + s.inv_kappa
    vol = float(np.prod(np.asarray(s.L, dtype=np.float32).astype(np.float64)))
    nm = int(np.prod(s.M))
    R = s.R[:, :3].astype(np.float64)
    V = s.V[:, :3].astype(np.float64)

    def force(R):
        counts, _ = oracle.density(R, s.T, s.L, s.M, s.K)
        phi = counts.astype(np.float64) / (2.0 ** 48 * (s.N / vol) * (vol / nm))
        Ff = oracle.gather_staggered(R, s.T, s.L, s.M, phi, A)
        Fb, _ = oracle.bonds(R, s.bonds, s.k_bond, s.r0, s.L)
        return Ff + Fb

    F = force(R)
    for _ in range(10):
        R, V = oracle.verlet_half1(R, V, F, s.dt, s.L)
        F = force(R)
        V = oracle.verlet_half2(V, F, s.dt)[0]
    Rg = by_tag(host(st.R)[:, :3].astype(np.float64), host(st.tag), s.N)
    d = np.abs(Rg - R)
    d = np.minimum(d, np.asarray(s.L) - d)
    assert d.max() / max(s.L) <= 1e-5
    assert hpf.hpf_get_device_status() == 0
    with pytest.raises(ValueError):
        st.step_fused()
