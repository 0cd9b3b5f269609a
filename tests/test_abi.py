"""The C-ABI library loads and exports every function include/hpf.h declares;
host-side argument checks reject bad input before anything is enqueued.
No GPU is needed: none of these calls reaches a kernel launch."""
import ctypes as C
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hpf():
    from paper_1310_2041_amd import build
    if build.is_stale():
        build.build()
    from paper_1310_2041_amd import hpf as h
    h.lib()
    return h


def test_exports_every_declared_function(hpf):
    declared = hpf.declared_functions()
    assert {"hpf_density_scatter", "hpf_field_potential", "hpf_field_gradient", "hpf_force_gather",
            "bond_forces", "verlet_step"} <= set(declared)
    out = subprocess.check_output(["nm", "-D", "--defined-only", hpf.LIB_PATH], text=True)
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    for f in declared:
        assert getattr(hpf.lib(), f) is not None


def test_abi_version_and_strings(hpf):
    L = hpf.lib()
    assert L.hpf_abi_version() == 1
    assert L.hpf_status_string(0) == b"ok"
    assert L.hpf_status_string(-1) == b"invalid argument"


def test_mesh_make(hpf):
    m = hpf.hpf_mesh_make((18.8, 18.8, 18.8), (20, 20, 20), 20000)
    assert list(m.M) == [20, 20, 20]
    import numpy as np
    assert m.s[0] == np.float32(20 / np.float64(np.float32(18.8)))
    assert m.c_norm == 8000 / (2.0 ** 48 * 20000)
    with pytest.raises(hpf.HpfError):
        hpf.hpf_mesh_make((18.8, 0.0, 18.8), (20, 20, 20), 1)
    with pytest.raises(hpf.HpfError):
        hpf.hpf_mesh_make((18.8, 18.8, 18.8), (20, 2, 20), 1)


def test_invalid_arguments_rejected_on_host(hpf):
    L = hpf.lib()
    m = hpf.hpf_mesh_make(10.0, 10, 100)
    dummy = C.c_void_p(0x1000)         # never dereferenced: checks fail first
    EINVAL = -1
    assert L.hpf_density_scatter(dummy, dummy, 10, C.byref(m), 0, dummy, None) == EINVAL
    assert L.hpf_density_scatter(dummy, dummy, 10, C.byref(m), 9, dummy, None) == EINVAL
    assert L.hpf_density_scatter(None, dummy, 10, C.byref(m), 2, dummy, None) == EINVAL
    assert L.hpf_density_scatter(dummy, dummy, -1, C.byref(m), 2, dummy, None) == EINVAL
    bad = hpf.Mesh()
    bad.L[:] = [10, 10, 10]
    bad.M[:] = [10, 10, 2]
    bad.s[:] = [1, 1, 1]
    assert L.hpf_density_scatter(dummy, dummy, 10, C.byref(bad), 2, dummy, None) == EINVAL
    f = hpf.make_field(2, 1.0, 10.0, [[0.0, 1.0], [1.0, 0.0]])
    f.K = 9
    assert L.hpf_field_potential(dummy, C.byref(m), C.byref(f), dummy, None, None, None) == EINVAL
    box = (C.c_float * 3)(10, 10, 10)
    badbox = (C.c_float * 3)(10, -1, 10)
    assert L.bond_forces(dummy, 10, dummy, 17, 1.0, 0.0, box, dummy, None, None) == EINVAL
    assert L.bond_forces(dummy, 10, dummy, 2, 1.0, 0.0, badbox, dummy, None, None) == EINVAL
    assert L.verlet_step(dummy, dummy, dummy, None, 10, 0.0, box, 1, None, None) == EINVAL
    assert L.verlet_step(dummy, dummy, dummy, None, 10, 0.03, box, 3, None, None) == EINVAL
    assert L.hpf_reduce_partials(dummy, 9, dummy, None) == EINVAL
    r_in, t_in, r_out, t_out = (C.c_void_p(0x1000 * k) for k in (2, 3, 4, 5))
    # in == out aliasing is rejected
    assert L.hpf_sort_by_cell(C.byref(m), 8, 10, r_in, None, t_in, None, None, 0, r_in, None,
                              t_out, None, None, None, dummy, 1 << 30, None) == EINVAL
    # too small or missing workspace
    assert L.hpf_sort_by_cell(C.byref(m), 8, 10, r_in, None, t_in, None, None, 0, r_out, None,
                              t_out, None, None, None, dummy, 16, None) == -3
    assert L.hpf_sort_by_cell(C.byref(m), 8, 10, r_in, None, t_in, None, None, 0, r_out, None,
                              t_out, None, None, None, None, 1 << 30, None) == -3
    # velocities given without an output buffer
    assert L.hpf_sort_by_cell(C.byref(m), 8, 10, r_in, dummy, t_in, None, None, 0, r_out, None,
                              t_out, None, None, None, dummy, 1 << 30, None) == EINVAL
    assert L.hpf_sort_workspace_bytes(10, C.byref(m), 17) == 0
    assert L.hpf_get_device_status(None, 0, None) == EINVAL
    r_n, v, g, cs = (C.c_void_p(0x1000 * k) for k in (6, 7, 8, 9))
    # hpf_advance_scatter / hpf_density_finish_cells: mesh limits, counts, workspace
    cnt, wk = C.c_void_p(0x10000), C.c_void_p(0x20000)
    m16 = hpf.hpf_mesh_make(16.0, 16, 100)
    need = L.hpf_scatter_workspace_bytes(10, C.byref(m16), 2, 8, 1)
    assert need > 0

    def advs(mesh=m16, counts=cnt, work=wk, nbytes=need, B=8, halo=1):
        return L.hpf_advance_scatter(r_in, r_n, v, t_in, 10, C.byref(mesh), 2, g, None, 0, 100.0, 0.0,
                                     box, None, 0.03, cs, B, halo, counts, work, nbytes, None, None, None,
                                     None, None)
    assert advs(mesh=m) == EINVAL                     # M = 10 < B + 1 + 2 halo
    assert advs(counts=None) == EINVAL
    assert advs(halo=3) == EINVAL
    assert advs(nbytes=need - 1) == -3
    assert advs(work=None) == -3
    # thermostat descriptions: probability outside [0, 1], no time level, no tags, kT <= 0
    for p, kT, step, tag in ((1.5, 1.0, 8, 9), (-0.1, 1.0, 8, 9), (0.5, 1.0, None, 9),
                             (0.5, 1.0, 8, None), (0.5, 0.0, 8, 9)):
        th = hpf.Thermostat()
        th.p, th.kT, th.seed = p, kT, 1
        th.step = None if step is None else 0x1000 * step
        th.tag = None if tag is None else 0x1000 * tag
        assert L.hpf_andersen(v, None, 10, C.byref(th), None, None) == EINVAL
        assert L.hpf_advance(r_in, r_n, v, t_in, 10, C.byref(m), 2, g, None, 0, 100.0, 0.0, box, None,
                             0.03, None, None, None, C.byref(th), None) == EINVAL
    assert L.hpf_andersen(v, None, 10, None, None, None) == EINVAL
    assert L.hpf_density_finish_cells(None, 10, C.byref(m16), 2, 8, 1, wk, need, None) == EINVAL
    assert L.hpf_density_finish_cells(cnt, 10, C.byref(m16), 2, 8, 1, wk, need - 1, None) == -3
    f2 = hpf.make_field(2, 1.0, 10.0, [[0.0, 1.0], [1.0, 0.0]])
    vv = C.c_void_p(0x30000)
    assert L.hpf_field_potential_cells(None, 10, C.byref(m16), C.byref(f2), 8, 1, wk, need, vv, None,
                                       None, None) == EINVAL
    assert L.hpf_field_potential_cells(cnt, 10, C.byref(m), C.byref(f2), 8, 1, wk, need, vv, None,
                                       None, None) == EINVAL                 # mesh too small for the boxes
    assert L.hpf_field_potential_cells(cnt, 10, C.byref(m16), C.byref(f2), 8, 1, wk, need - 1, vv, None,
                                       None, None) == -3


def test_sort_workspace_size(hpf):
    m = hpf.hpf_mesh_make(149.4, 128, 10_000_000)
    n = hpf.hpf_sort_workspace_bytes(10_000_000, m, 8)
    nk = hpf.sort_key_count(m, 8)
    assert nk == 16 ** 3                      # one key per brick of 8^3 cells
    assert n >= 3 * 4 * 10_000_000 + 2 * 4 * (nk + 2)


def test_static_scatter_refuses_problems_beyond_its_scratch(hpf):
    """hpf_density_scatter_cells_static holds its scratch in a fixed 32 MiB device array:
    10M beads on a 128^3 mesh need 184 MB and are refused on the host (HPF_ETOOBIG)
    before anything is enqueued; bad arguments still give HPF_EINVAL."""
    L = hpf.lib()
    m = hpf.hpf_mesh_make(149.4, 128, 10_000_000)
    need = L.hpf_scatter_workspace_bytes(10_000_000, C.byref(m), 2, 8, 2)
    assert need > hpf.HPF_STATIC_SCRATCH_BYTES == 32 << 20
    dummy = C.c_void_p(0x1000)         # never dereferenced: checks fail first
    assert L.hpf_density_scatter_cells_static(dummy, dummy, 10_000_000, C.byref(m), 2, dummy, 8, 2,
                                              dummy, None) == hpf.HPF_ETOOBIG
    assert L.hpf_density_scatter_cells_static(dummy, dummy, 10_000_000, C.byref(m), 2, None, 8, 2,
                                              dummy, None) == -1
    assert L.hpf_status_string(hpf.HPF_ETOOBIG).startswith(b"problem exceeds")
