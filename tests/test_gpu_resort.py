"""GPU: the incremental re-sort (hpf_resort_by_cell) gives exactly the order of the full
counting sort (hpf_sort_by_cell) and of the oracle's (brick, tag) permutation, from the
order of an earlier sort after the beads have moved: few or all beads changing brick,
bricks whose movers overflow the LDS sort, beads becoming unbinnable and binnable again,
16-cell bricks and the full 10M-bead blend. A broken precondition raises the flag and
leaves a set of valid indices."""
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


def _moved(s, B, steps, halo=1):
    """A system sorted once and then moved `steps` fused steps without sorting."""
    st = engine.HpfState.from_system(s, sort_brick=B, halo=halo)
    st.start(sort=True)
    st.prime()
    if steps:
        st.run_fused(steps, report_every=0, sort_every=0)
    torch.cuda.synchronize()
    return st


def _sorts(st):
    """(R, Vel, T, tag, bonds, cell_start) after the re-sort and after the full sort, both
    from the state's current arrays and order."""
    D = st.bonds.shape[0]
    out = []
    for resort in (True, False):
        R2, V2, T2, g2 = (torch.empty_like(x) for x in (st.R, st.Vel, st.T, st.tag))
        b2 = torch.empty_like(st.bonds)
        cs = torch.full_like(st.cell_start, -7)
        args = (st.mesh, st.B, st.R, st.Vel, st.T, st.tag, st.bonds if D else None, R2, V2, T2, g2,
                b2 if D else None, st.work)
        if resort:
            hpf.hpf_resort_by_cell(*args, st.cell_start, cs)
        else:
            hpf.hpf_sort_by_cell(*args, cell_start=cs)
        out.append(tuple(host(x) for x in (R2, V2, T2, g2, b2, cs)))
    return out


def _bits_equal(a, b):
    """Bitwise equality of two tuples of arrays (NaN positions included)."""
    return all(np.array_equal(np.ascontiguousarray(x).view(np.uint8), np.ascontiguousarray(y).view(np.uint8))
               for x, y in zip(a, b))


def _check_equal_and_oracle(st, s):
    a, b = _sorts(st)
    assert _bits_equal(a, b)
    # the oracle's order of the current positions (tags are the original indices)
    R = host(st.R)
    tag = host(st.tag)
    perm, _ = oracle.sort_perm(R, tag, s.L, s.M, st.B)
    assert np.array_equal(a[3], tag[perm])
    assert np.array_equal(a[0], R[perm])


CASES = [
    ("c1_b8", lambda: wl.build(wl.SPECS["c1"]), 8, 15),
    ("ragged_k3_b3", lambda: wl.small_system(300, 10, (13.7, 15.1, 14.2), (13, 15, 14), K=3, seed=5,
                                             n_solvent=700), 3, 9),
    ("b4", lambda: wl.small_system(500, 12, 16.0, 15, seed=9), 4, 25),
    ("b16", lambda: wl.small_system(1500, 12, 26.1, (24, 23, 26), seed=64), 16, 12),
]


@pytest.mark.parametrize("name,make,B,steps", CASES, ids=[c[0] for c in CASES])
def test_resort_equals_full_sort_and_oracle(name, make, B, steps):
    s = make()
    st = _moved(s, B, steps, halo=1 if B > 3 else 0)
    hpf.hpf_get_device_status(clear=True)
    _check_equal_and_oracle(st, s)
    assert hpf.hpf_get_device_status() == 0


def test_resort_when_every_bead_moves_and_buckets_overflow_lds():
    """Positions redrawn uniformly after the sort: nearly every bead changes brick, and with
    40,000 beads in 8 bricks a brick receives more movers than the LDS sort holds."""
    s = wl.small_system(4000, 10, 18.0, 16, seed=17)
    st = _moved(s, 8, 0)
    rng = np.random.default_rng(3)
    st.R.copy_(dev(wl.wrap_f32(rng.random((s.N, 3)) * 18.0, (18.0,) * 3), torch.float32))
    hpf.hpf_get_device_status(clear=True)
    _check_equal_and_oracle(st, s)
    assert hpf.hpf_get_device_status() == 0


def test_resort_beads_leaving_and_entering_the_unbinned_tail():
    """Beads that cannot be binned sort last; beads go there and come back between sorts."""
    s = wl.build(wl.SPECS["c1"])
    s.R[[3, 500, 7000]] = np.nan                      # unbinnable at the first sort
    st = _moved(s, 8, 0)
    R = host(st.R)
    tag = host(st.tag)
    back = np.isin(tag, [3, 500, 7000])
    R[back] = np.float32(1.25)                          # binnable again
    R[[10, 11, 4000, 19999]] = np.nan                   # newly unbinnable
    st.R.copy_(dev(R, torch.float32))
    hpf.hpf_get_device_status(clear=True)
    a, b = _sorts(st)
    assert _bits_equal(a, b)
    nk = hpf.sort_key_count(st.mesh, 8)
    unbinned = int((~np.isfinite(R)).any(axis=1).sum())    # the chains' neighbours went NaN too
    assert unbinned >= 4 and a[5][nk + 1] - a[5][nk] == unbinned
    assert not np.isfinite(a[0][-unbinned:]).all(axis=1).any()
    hpf.hpf_get_device_status(clear=True)


def test_resort_of_the_10m_blend_after_20_steps():
    """The benchmark's system (16-cell bricks) after 20 fused steps: the re-sort equals the
    full sort bit for bit."""
    s = wl.build(wl.SPECS["c3"])
    st = _moved(s, 0, 20, halo=2)
    del s
    assert st.B == 16
    a, b = _sorts(st)
    assert _bits_equal(a, b)
    assert hpf.hpf_get_device_status() == 0


def test_resort_flags_an_input_out_of_order():
    """Two beads of one brick swapped after the sort break the precondition: the flag is
    raised and every index written stays a real input row."""
    s = wl.small_system(300, 10, 12.0, 12, seed=44)
    st = _moved(s, 4, 3)
    cs = host(st.cell_start)
    k = int(np.argmax(np.diff(cs[:-1])))                # the fullest brick
    i, j = int(cs[k]), int(cs[k]) + 1
    for x in (st.R, st.Vel, st.T, st.tag):
        t = x[i].clone()
        x[i] = x[j]
        x[j] = t
    hpf.hpf_get_device_status(clear=True)
    a, _ = _sorts(st)
    assert hpf.hpf_get_device_status(clear=True) & hpf.HPF_FLAG_SORT_ORDER
    assert np.isin(a[0][:, 0], host(st.R)[:, 0]).all()
    assert ((a[4] >= -1) & (a[4] < s.N)).all()


def test_stepping_with_resorts_equals_full_sorts():
    """30 fused steps of the 20,000-bead melt with a sort every 5: re-sorting from the last
    order and sorting from scratch move every bead identically and keep the same order."""
    s = wl.build(wl.SPECS["c1"])
    a = engine.HpfState.from_system(s)
    b = engine.HpfState.from_system(s)
    a.resort, b.resort = True, False
    for st in (a, b):
        st.start(sort=True)
        st.prime()
        st.run_fused(30, report_every=0, sort_every=5)
    for x, y in zip(a.host_beads(), b.host_beads()):
        assert np.array_equal(x, y)
    assert np.array_equal(host(a.cell_start), host(b.cell_start))
    assert hpf.hpf_get_device_status() == 0
