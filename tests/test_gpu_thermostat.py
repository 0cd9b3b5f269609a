"""GPU: the Andersen thermostat (Integration methods section, NVT) against the oracle.

Collision decisions are integers drawn from the counter-based generator keyed on
(tag, time level), so they must agree with the oracle's exactly: a bead that
collides on one side and not on the other would differ by a whole thermal
velocity. New velocities agree to FP32 rounding of Box-Muller (<= 1e-6 of the
largest speed). The thermostat inside the fused passes and the batch must
move every bead bit for bit as the separate calls do.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import dev, host  # noqa: E402
from paper_1310_2041_amd import engine, hpf  # noqa: E402
from synth import workloads as wl  # noqa: E402


@pytest.mark.parametrize("p,kT,step", [(0.5, 2.0, 7), (1.0, 1.0, 123456789012), (0.03, 0.5, 1)])
def test_andersen_matches_oracle(p, kT, step):
    n = 300_007
    rng = np.random.default_rng(5)
    V = np.zeros((n, 3), np.float32)
    V[:, :3] = rng.standard_normal((n, 3)).astype(np.float32)
    tag = rng.permutation(n).astype(np.int32)
    im = rng.uniform(0.5, 2.0, n).astype(np.float32)
    want, mask = oracle.andersen(V, tag, kT, p, 0xDEADBEEF12345, step, inv_mass=im)
    Vd, tagd, imd = dev(V, torch.float32), dev(tag, torch.int32), dev(im, torch.float32)
    tstep = torch.tensor([step], dtype=torch.int64, device="cuda")
    th = hpf.make_thermostat(p, kT, 0xDEADBEEF12345, tstep, tagd)
    part = torch.zeros((4, hpf.HPF_NPART), dtype=torch.float64, device="cuda")
    hpf.hpf_andersen(Vd, th, inv_mass=imd, kin_part=part)
    got = host(Vd)[:, :3].astype(np.float64)
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"p={p}: {mask.mean():.4f} collided, max rel error {err:.2e}")
    assert err <= 1e-6
    assert np.array_equal(got[mask == 0], V[mask == 0, :3].astype(np.float64))
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    hpf.hpf_reduce_partials(part, 4, out)
    ke = (0.5 / im.astype(np.float64) * (want ** 2).sum(1)).sum()
    assert host(out)[0] == pytest.approx(ke, rel=1e-6)


def test_thermostat_six_calls_follow_oracle():
    """20 steps of the 20,000-bead melt at collision probability 0.3 per step (rate 10):
    energies within 1e-4 of the oracle's NVT run at every step."""
    s = wl.build(wl.SPECS["c1"])
    st = engine.HpfState.from_system(s)
    st.set_thermostat(10.0, seed=99)
    st.start(sort=True)
    trace = st.run(20, report_every=1, sort_every=7)
    Eg = np.array([[e["KE"], e["E_bond"], e["W"], e["E_tot"]] for e in trace])
    _, _, Eo = oracle.run_nvt(s, 20, 1, 1.0, np.float32(0.3), 99)
    rel = np.abs(Eg - Eo[1:]) / np.abs(Eo[1:])
    print("max rel diff (KE, Eb, W, Etot):", rel.max(0))
    assert rel.max() <= 1e-4
    assert hpf.hpf_get_device_status() == 0


@pytest.mark.parametrize("field_every", [1, 3])
@pytest.mark.parametrize("advance", ["scatter", "plain"])
def test_thermostat_fused_equals_six_calls_bitwise(advance, field_every):
    s = wl.build(wl.SPECS["c1"])
    a = engine.HpfState.from_system(s, field_every=field_every)
    a.set_thermostat(5.0, seed=7)
    a.start(sort=True)
    Ea = a.run(24, report_every=1, sort_every=6)
    a.prime()
    b = engine.HpfState.from_system(s, field_every=field_every, advance=advance)
    b.set_thermostat(5.0, seed=7)
    b.start(sort=True)
    b.prime()
    Eb = b.run_fused(24, report_every=1, sort_every=6)
    for x, y in zip(a.host_beads(), b.host_beads()):
        assert np.array_equal(x, y)
    for ea, eb in zip(Ea, Eb):
        for key in ("KE", "E_bond", "W"):
            assert eb[key] == pytest.approx(ea[key], rel=1e-12)
    assert hpf.hpf_get_device_status() == 0


def test_thermostat_graph_replays_draw_fresh_numbers():
    """A graph of 4 fused steps replayed 3 times equals 12 eager steps bit for bit: the time
    level is read on the device, so every replay draws new collisions."""
    s = wl.build(wl.SPECS["c1"])
    a = engine.HpfState.from_system(s)
    b = engine.HpfState.from_system(s)
    for st in (a, b):
        st.set_thermostat(5.0, seed=3)
        st.start(sort=True)
        st.prime()
    a.run_fused(12, report_every=0, sort_every=2)
    g = engine.Graph(lambda: b.run_fused(4, report_every=0, sort_every=2))
    for _ in range(3):
        g.launch()
    torch.cuda.synchronize()
    for x, y in zip(a.host_beads(), b.host_beads()):
        assert np.array_equal(x, y)
    assert int(host(a.tstep)[0]) == int(host(b.tstep)[0]) == 13
    del g


def test_batch_thermostat_matches_single_systems():
    """A batch with the thermostat moves every replica as its single-system run. The batch's
    tags are global (replica r's start at its first bead); the single system keeps the tags
    0..N_r-1 that its sort needs and offsets them in the generator's counter instead."""
    specs = [(40, 10, 13.3, 13, 0.0), (150, 10, 17.1, 16, 0.7), (60, 20, 15.5, 14, 2.0)]
    systems = [wl.small_system(nc, cl, L, M, seed=200 + i, chi_ab=chi)
               for i, (nc, cl, L, M, chi) in enumerate(specs)]
    b = engine.BatchState(systems, sort_every=5, thermostat_rate=4.0, thermostat_seed=11)
    b.start()
    b.step(12, report_last=True)
    off = 0
    for r, s in enumerate(systems):
        st = engine.HpfState.from_system(s)
        st.set_thermostat(4.0, seed=11, tag_offset=off)
        st.start(sort=True)
        st.prime()
        st.run_fused(12, report_every=0, sort_every=5)
        R, V, T, tag, bonds = st.host_beads()
        bR, bV, bT, btag, bbonds = b.replica_beads(r)
        assert np.array_equal(bR, R) and np.array_equal(bV, V)
        assert np.array_equal(btag, tag)
        off += s.N
    assert hpf.hpf_get_device_status() == 0
