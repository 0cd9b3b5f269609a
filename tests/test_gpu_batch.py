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
    """Tuning (which also varies the sort interval) moves every bead as untuned stepping does;
    compared by tag, since the storage order between sorts depends on the sort interval. A
    second tuning of the same replica set comes from the cache, without trials."""
    systems = _replicas()
    a = engine.BatchState(systems, sort_every=5)
    b = engine.BatchState(systems, sort_every=5)
    a.start()
    b.start()
    chosen, times = a.tune(trial_steps=20)
    assert len(times) == 14 and all(t > 0 for t in times)
    assert chosen["halo"] in (1, 2) and chosen["fuse_deposit"] in (0, 1)
    assert chosen["sort_every"] in (5, 10, 20, 30, 40)
    # per halo: the fused deposit with sort intervals 5, 10, 20, 30, 40 and the separate
    # scatter with two chunk sizes (sort every 10); each trial runs at least 20 steps,
    # rounded up to whole sort intervals, three times
    per_halo = sum(-(-20 // se) * se for se in (5, 10, 20, 30, 40)) + 2 * 20
    b.step(2 * per_halo * 3, report_last=False)
    for r in range(len(systems)):
        ra, rb = a.replica_beads(r), b.replica_beads(r)
        ta, tb = ra[3], rb[3]
        for x, y in zip(ra[:3], rb[:3]):
            assert np.array_equal(x[np.argsort(ta)], y[np.argsort(tb)])
    c = engine.BatchState(systems, sort_every=5)
    c.start()
    chosen2, times2 = c.tune(trial_steps=20)
    assert times2 == [] and chosen2 == chosen


def test_batch_rejects_small_meshes():
    s = wl.small_system(20, 10, 10.0, 10, seed=1)
    with pytest.raises(ValueError):
        engine.BatchState([s])


def _replica_counts(b, counts, r):
    """Replica r's block of a batch counts tensor as uint64 [K, Mz, My, Mx]."""
    off = b.K * sum(b.nm[:r])
    M = tuple(b.reps[r].M)
    blk = counts[off:off + b.K * b.nm[r]].cpu().numpy().view(np.uint64)
    return blk.reshape(b.K, M[2], M[1], M[0])


def _by_tag(arr, tag):
    out = np.zeros_like(arr)
    out[tag] = arr
    return out


def test_batch_density_matches_oracle():
    """hpf_batch_density: every replica's counts at the current positions bit-exact against
    the oracle, after the start (plain cell scatter) and after fused steps (the pending
    deposit finished into the output), and the batch steps on unchanged."""
    systems = _replicas()
    b = engine.BatchState(systems, sort_every=5)
    ref = engine.BatchState(systems, sort_every=5)
    b.start()
    ref.start()
    for n in (0, 7):
        if n:
            b.step(n, report_last=True)
            ref.step(n, report_last=True)
        out = b.density()
        for r, s in enumerate(systems):
            R, _, T, tag, _ = b.replica_beads(r)
            want, sk = oracle.density(_by_tag(R, tag), _by_tag(T, tag), s.L, s.M, s.K)
            assert sk == 0
            assert np.array_equal(_replica_counts(b, out, r), want), (n, r)
    b.step(3, report_last=True)
    ref.step(3, report_last=True)
    for r in range(len(systems)):
        for x, y in zip(b.replica_beads(r), ref.replica_beads(r)):
            assert np.array_equal(x, y)
    assert hpf.hpf_get_device_status() == 0


def test_batch_rejects_bond_into_another_replica():
    systems = _replicas()[:2]
    systems[0].bonds[0, 3] = systems[0].N + 2        # a partner inside replica 1
    with pytest.raises(hpf.HpfError):
        engine.BatchState(systems)


@pytest.mark.slow
def test_full_size_64_replica_sweep_sampled():
    """The 64-replica sweep at full size (6.8M beads) in the benchmark's launch shape (one
    batch, 20 steps per HIP graph). For replicas 0, 31 and 63: the counts at the current
    positions bit-exact against the oracle after the start and after a replay (the pending
    fused deposit), the step-0 forces (from the first half kick) within 1e-5 and the
    step-0 energies of the oracle; after the replay each equals its single-system run bit
    for bit."""
    systems = [wl.build_replica(sp, r) for r, sp in enumerate(wl.replica_specs())]
    b = engine.BatchState(systems, sort_every=10)
    b.start()
    E0 = b.energies()
    out = b.density()
    for r in (0, 31, 63):
        s = systems[r]
        _, _, Eo = oracle.run(s, 0)
        assert E0[r, 0] == pytest.approx(Eo[0, 0], rel=1e-12)        # KE
        assert E0[r, 1] == pytest.approx(Eo[0, 1], rel=1e-6)         # E_bond (FP32 terms)
        assert E0[r, 2] == pytest.approx(Eo[0, 2], rel=1e-9)         # W
        R, V, T, tag, _ = b.replica_beads(r)
        want, _ = oracle.density(_by_tag(R, tag), s.T, s.L, s.M, s.K)
        assert np.array_equal(_replica_counts(b, out, r), want), r
        # v_1/2 = v_0 + dt/2 F(x_0): the step-0 force from the batched kernels
        Ff, Fb, _ = oracle.forces(s)
        F_gpu = (_by_tag(V, tag)[:, :3].astype(np.float64) - s.V[:, :3]) / (0.5 * s.dt)
        err = np.abs(F_gpu - (Ff + Fb)).max() / np.abs(Ff + Fb).max()
        assert err <= 1e-5, (r, err)
    del out
    torch.cuda.synchronize()
    g = engine.Graph(lambda: b.step(20, report_last=True))
    g.launch()
    torch.cuda.synchronize()
    out = b.density()
    for r in (0, 31, 63):
        R, _, T, tag, _ = b.replica_beads(r)
        want, _ = oracle.density(_by_tag(R, tag), systems[r].T, systems[r].L, systems[r].M,
                                 systems[r].K)
        assert np.array_equal(_replica_counts(b, out, r), want), r
        st, _ = _single(systems[r], 20, 10)
        for x, y in zip(b.replica_beads(r), st.host_beads()):
            assert np.array_equal(x, y), f"replica {r}"
    assert hpf.hpf_get_device_status() == 0
    del g
