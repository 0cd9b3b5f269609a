"""Batched replicas, HIP-graph replay and the autotuner on the GPU.

The batch must move every replica's beads exactly as the single-system calls
do (bit for bit; FP64 energy sums only regroup), graph replays must equal
eager stepping on every replay, and tuning must not perturb trajectories.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_1310_2041_amd import engine, hpf  # noqa: E402
from synth import workloads as wl  # noqa: E402


def _replicas():
    specs = [(40, 10, 13.3, 13, 0.0), (150, 10, 17.1, 16, 0.7), (60, 20, 15.5, 14, 2.0),
             (33, 10, (13.7, 15.1, 14.2), (13, 15, 14), 1.3), (220, 10, 20.9, 21, 1.0)]
    out = []
    for i, (nc, cl, L, M, chi) in enumerate(specs):
        s = wl.small_system(nc, cl, L, M, seed=100 + i, chi_ab=chi)
        out.append(s)
    return out


def _single(s, steps, sort_every):
    st = engine.HpfState.from_system(s)
    st.start(sort=True)
    st.prime()
    e = st.run_fused(steps, report_every=steps, sort_every=sort_every)
    return st, e[-1]


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("bead_chunk,mesh_chunk,halo", [(512, 2048, 1), (4096, 16384, 2)])
def test_batch_matches_single_systems_bitwise(bead_chunk, mesh_chunk, halo, fuse):
    systems = _replicas()
    steps, sort_every = 12, 5
    b = engine.BatchState(systems, sort_every=sort_every, halo=halo, bead_chunk=bead_chunk,
                          mesh_chunk=mesh_chunk, fuse_deposit=fuse)
    b.start()
    b.step(steps, report_last=True)
    E = b.energies()
    for r, s in enumerate(systems):
        st, e1 = _single(s, steps, sort_every)
        for x, y in zip(b.replica_beads(r), st.host_beads()):
            assert np.array_equal(x, y), f"replica {r}"
        for j, key in enumerate(["KE", "E_bond", "W"]):
            assert E[r, j] == pytest.approx(e1[key], rel=1e-12, abs=1e-9)
        assert E[r, 3] == pytest.approx(e1["E_tot"], rel=1e-12)
    assert hpf.hpf_get_device_status() == 0


def test_batch_graph_replays_match_eager():
    systems = _replicas()
    a = engine.BatchState(systems, sort_every=5)
    b = engine.BatchState(systems, sort_every=5)
    a.start()
    b.start()
    torch.cuda.synchronize()
    g = engine.Graph(lambda: a.step(10, report_last=True))
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        b.step(10, report_last=True)
        torch.cuda.synchronize()
        for r in range(len(systems)):
            for x, y in zip(a.replica_beads(r), b.replica_beads(r)):
                assert np.array_equal(x, y), f"replay {rep} replica {r}"
        assert np.array_equal(a.energies(), b.energies())
    del g


def test_graph_of_single_system_steps_matches_eager():
    s = wl.build(wl.SPECS["c1"])
    a = engine.HpfState.from_system(s)
    b = engine.HpfState.from_system(s)
    for st in (a, b):
        st.start(sort=True)
        st.prime()
    torch.cuda.synchronize()

    def ten():
        for _ in range(10):
            a.step_fused(report=False, sort=a.steps_done % 5 == 0)

    g = engine.Graph(ten)
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        b.run_fused(10, report_every=0, sort_every=5)
        torch.cuda.synchronize()
        for x, y in zip(a.host_beads(), b.host_beads()):
            assert np.array_equal(x, y), f"replay {rep}"
    del g


def test_batch_tune_keeps_trajectories():
    systems = _replicas()
    a = engine.BatchState(systems, sort_every=5)
    b = engine.BatchState(systems, sort_every=5)
    a.start()
    b.start()
    chosen, times = a.tune(trial_steps=2)
    assert len(times) == 20 and all(t > 0 for t in times)
    assert chosen["halo"] in (1, 2) and chosen["fuse_deposit"] in (0, 1)
    b.step(len(times) * 3, report_last=False)
    for r in range(len(systems)):
        for x, y in zip(a.replica_beads(r), b.replica_beads(r)):
            assert np.array_equal(x, y)


def test_batch_rejects_small_meshes():
    s = wl.small_system(20, 10, 10.0, 10, seed=1)
    with pytest.raises(ValueError):
        engine.BatchState([s])


@pytest.mark.slow
def test_full_size_64_replica_sweep_sampled():
    """The 64-replica sweep at full size (6.8M beads) in the benchmark's launch shape (one
    batch, 20 steps per HIP graph): the step-0 energies of sampled replicas match the oracle,
    and after a replay replicas 0, 31 and 63 equal their single-system runs bit for bit."""
    systems = [wl.build_replica(sp, r) for r, sp in enumerate(wl.replica_specs())]
    b = engine.BatchState(systems, sort_every=10)
    b.start()
    E0 = b.energies()
    for r in (0, 31, 63):
        _, _, Eo = oracle.run(systems[r], 0)
        assert E0[r, 0] == pytest.approx(Eo[0, 0], rel=1e-12)        # KE
        assert E0[r, 1] == pytest.approx(Eo[0, 1], rel=1e-6)         # E_bond (FP32 terms)
        assert E0[r, 2] == pytest.approx(Eo[0, 2], rel=1e-9)         # W
    torch.cuda.synchronize()
    g = engine.Graph(lambda: b.step(20, report_last=True))
    g.launch()
    torch.cuda.synchronize()
    for r in (0, 31, 63):
        st, _ = _single(systems[r], 20, 10)
        for x, y in zip(b.replica_beads(r), st.host_beads()):
            assert np.array_equal(x, y), f"replica {r}"
    assert hpf.hpf_get_device_status() == 0
    del g
