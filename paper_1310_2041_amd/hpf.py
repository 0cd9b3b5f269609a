"""Python binding of libhpf (include/hpf.h): argument marshalling only.

Every function here has the name of the C entry point it calls, takes torch
tensors that live on the GPU (plus host-side parameter structs), checks
dtypes, shapes and contiguity, and passes raw device pointers and the current
HIP stream to the library. All arithmetic happens in the library's kernels.
If the library is not built, importing this module raises; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# HPF_LIBRARY names another build of the same library (for comparing builds); the
# in-tree one is the default.
LIB_PATH = os.environ.get("HPF_LIBRARY") or os.path.join(_HERE, "libhpf.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hpf.h")

HPF_FIX_BITS = 16
HPF_MAX_TYPES = 8
HPF_NPART = 4096
HPF_MAX_BONDS = 16

HPF_FLAG_BAD_BEAD = 0x1
HPF_FLAG_OVERFLOW = 0x2
HPF_FLAG_NONFINITE = 0x4
HPF_FLAG_BAD_BOND = 0x8
HPF_FLAG_SORT_ORDER = 0x10

HPF_ETOOBIG = -4
HPF_STATIC_SCRATCH_BYTES = 32 << 20


class HpfError(RuntimeError):
    def __init__(self, fn: str, status: int, text: str):
        super().__init__(f"{fn} failed: {text} (status {status})")
        self.status = status


class Mesh(C.Structure):
    """hpf_mesh_t"""
    _fields_ = [("L", C.c_float * 3), ("M", C.c_int32 * 3), ("s", C.c_float * 3),
                ("reserved", C.c_int32), ("c_norm", C.c_double)]


class Field(C.Structure):
    """hpf_field_t"""
    _fields_ = [("K", C.c_int32), ("reserved", C.c_int32), ("kT", C.c_double),
                ("inv_kappa", C.c_double), ("chi", C.c_double * (HPF_MAX_TYPES * HPF_MAX_TYPES))]


class Replica(C.Structure):
    """hpf_replica_t"""
    _fields_ = [("bead_offset", C.c_int64), ("n_beads", C.c_int64), ("L", C.c_float * 3),
                ("M", C.c_int32 * 3), ("kT", C.c_double), ("inv_kappa", C.c_double),
                ("chi", C.c_double * (HPF_MAX_TYPES * HPF_MAX_TYPES))]


class BatchConfig(C.Structure):
    """hpf_batch_config_t"""
    _fields_ = [("K", C.c_int32), ("D", C.c_int32), ("k_bond", C.c_float), ("r0", C.c_float),
                ("dt", C.c_float), ("brick", C.c_int32), ("halo", C.c_int32),
                ("sort_every", C.c_int32), ("bead_chunk", C.c_int32), ("mesh_chunk", C.c_int32),
                ("fuse_deposit", C.c_int32), ("thermo_p", C.c_float), ("reserved", C.c_int32),
                ("thermo_seed", C.c_uint64)]


class Thermostat(C.Structure):
    """hpf_thermostat_t (step and tag are device pointers)"""
    _fields_ = [("p", C.c_float), ("kT", C.c_float), ("seed", C.c_uint64), ("step", C.c_void_p),
                ("tag", C.c_void_p), ("tag_offset", C.c_int64)]


def make_thermostat(p: float, kT: float, seed: int, step, tag, tag_offset: int = 0) -> Thermostat:
    """Andersen thermostat description: collision probability p per step, bath kT, generator
    key seed; step is a device int64 tensor of one element (the time level), tag the beads'
    int32 tags in storage order; tag_offset is added to every tag in the generator's counter."""
    th = Thermostat()
    th.p = float(p)
    th.kT = float(kT)
    th.seed = int(seed)
    th.step = _dev(step, "step", torch.int64, (1,))
    th.tag = _dev(tag, "tag", torch.int32, None)
    th.tag_offset = int(tag_offset)
    return th


class BatchBuffers(C.Structure):
    """hpf_batch_buffers_t"""
    _fields_ = [("R", C.c_void_p * 2), ("Vel", C.c_void_p * 2), ("T", C.c_void_p * 2),
                ("tag", C.c_void_p * 2), ("bonds", C.c_void_p * 2), ("counts", C.c_void_p),
                ("V", C.c_void_p), ("G", C.c_void_p)]


_lib = None
_P = C.c_void_p

_SIGNATURES = {
    "hpf_abi_version": ([], C.c_int32),
    "hpf_status_string": ([C.c_int32], C.c_char_p),
    "hpf_mesh_make": ([_P, _P, C.c_int64, C.POINTER(Mesh)], C.c_int32),
    "hpf_density_scatter": ([_P, _P, C.c_int64, C.POINTER(Mesh), C.c_int32, _P, _P], C.c_int32),
    "hpf_scatter_workspace_bytes": ([C.c_int64, C.POINTER(Mesh), C.c_int32, C.c_int32, C.c_int32],
                                    C.c_size_t),
    "hpf_density_scatter_cells": ([_P, _P, C.c_int64, C.POINTER(Mesh), C.c_int32, _P, C.c_int32,
                                   C.c_int32, _P, _P, C.c_size_t, _P], C.c_int32),
    "hpf_density_scatter_cells_static": ([_P, _P, C.c_int64, C.POINTER(Mesh), C.c_int32, _P, C.c_int32,
                                          C.c_int32, _P, _P], C.c_int32),
    "hpf_field_potential": ([_P, C.POINTER(Mesh), C.POINTER(Field), _P, _P, _P, _P], C.c_int32),
    "hpf_field_gradient": ([_P, C.POINTER(Mesh), C.c_int32, _P, _P, _P], C.c_int32),
    "hpf_force_gather": ([_P, _P, C.c_int64, C.POINTER(Mesh), C.c_int32, _P, _P, _P], C.c_int32),
    "hpf_force_gather_staggered": ([_P, _P, C.c_int64, C.POINTER(Mesh), C.c_int32, _P, _P, _P],
                                   C.c_int32),
    "bond_forces": ([_P, C.c_int64, _P, C.c_int32, C.c_float, C.c_float, _P, _P, _P, _P],
                    C.c_int32),
    "angle_forces": ([_P, C.c_int64, _P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P, _P, _P],
                     C.c_int32),
    "hpf_sort_angles": ([C.POINTER(Mesh), C.c_int32, C.c_int64, _P, C.c_int32, _P, _P, C.c_size_t, _P],
                        C.c_int32),
    "verlet_step": ([_P, _P, _P, _P, C.c_int64, C.c_float, _P, C.c_int32, _P, _P], C.c_int32),
    "hpf_reduce_partials": ([_P, C.c_int32, _P, _P], C.c_int32),
    "hpf_advance": ([_P, _P, _P, _P, C.c_int64, C.POINTER(Mesh), C.c_int32, _P, _P, C.c_int32,
                     C.c_float, C.c_float, _P, _P, C.c_float, _P, _P, _P, _P, _P], C.c_int32),
    "hpf_andersen": ([_P, _P, C.c_int64, _P, _P, _P], C.c_int32),
    "hpf_advance_scatter": ([_P, _P, _P, _P, C.c_int64, C.POINTER(Mesh), C.c_int32, _P, _P, C.c_int32,
                             C.c_float, C.c_float, _P, _P, C.c_float, _P, C.c_int32, C.c_int32, _P, _P,
                             C.c_size_t, _P, _P, _P, _P, _P], C.c_int32),
    "hpf_density_finish_cells": ([_P, C.c_int64, C.POINTER(Mesh), C.c_int32, C.c_int32, C.c_int32,
                                  _P, C.c_size_t, _P], C.c_int32),
    "hpf_field_potential_cells": ([_P, C.c_int64, C.POINTER(Mesh), C.POINTER(Field), C.c_int32, C.c_int32,
                                   _P, C.c_size_t, _P, _P, _P, _P], C.c_int32),
    "hpf_sort_workspace_bytes": ([C.c_int64, C.POINTER(Mesh), C.c_int32], C.c_size_t),
    "hpf_sort_by_cell": ([C.POINTER(Mesh), C.c_int32, C.c_int64, _P, _P, _P, _P, _P, C.c_int32,
                          _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P], C.c_int32),
    "hpf_resort_by_cell": ([C.POINTER(Mesh), C.c_int32, C.c_int64, _P, _P, _P, _P, _P, C.c_int32,
                            _P, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P], C.c_int32),
    "hpf_get_device_status": ([C.POINTER(C.c_uint32), C.c_int32, _P], C.c_int32),
    "hpf_batch_workspace_bytes": ([C.POINTER(Replica), C.c_int32, C.POINTER(BatchConfig)],
                                  C.c_size_t),
    "hpf_batch_create": ([C.POINTER(Replica), C.c_int32, C.POINTER(BatchConfig),
                          C.POINTER(BatchBuffers), _P, C.c_size_t, C.POINTER(C.c_void_p)],
                         C.c_int32),
    "hpf_batch_start": ([_P, _P], C.c_int32),
    "hpf_batch_step": ([_P, C.c_int32, C.c_int32, _P], C.c_int32),
    "hpf_batch_current": ([_P, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                           C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                           C.POINTER(C.c_void_p)], C.c_int32),
    "hpf_batch_density": ([_P, _P, _P], C.c_int32),
    "hpf_batch_tune": ([_P, C.c_int32, _P, C.POINTER(BatchConfig), C.POINTER(C.c_float),
                        C.POINTER(C.c_int32)], C.c_int32),
    "hpf_batch_destroy": ([_P], C.c_int32),
    "hpf_graph_begin": ([_P], C.c_int32),
    "hpf_graph_end": ([_P, C.POINTER(C.c_void_p)], C.c_int32),
    "hpf_graph_launch": ([_P, _P], C.c_int32),
    "hpf_graph_destroy": ([_P], C.c_int32),
}


def lib():
    """Load libhpf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1310_2041_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        if L.hpf_abi_version() != 1:
            raise ImportError("libhpf ABI version mismatch")
        _lib = L
    return _lib


def declared_functions() -> list:
    """Names of the functions declared in include/hpf.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(\w+)\s*\([^;{]*\)\s*;", text)) -
                  {"if", "while", "for", "return", "sizeof"})


def _check(fn: str, status: int):
    if status != 0:
        raise HpfError(fn, status, lib().hpf_status_string(status).decode())


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _dev(t: torch.Tensor | None, name: str, dtype=None, shape=None, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr()) if t.numel() else None


_U64 = (torch.int64, torch.uint64) if hasattr(torch, "uint64") else (torch.int64,)


def hpf_mesh_make(L, M, n_beads: int) -> Mesh:
    Lf = (C.c_float * 3)(*[float(x) for x in (L if hasattr(L, "__len__") else (L,) * 3)])
    Mi = (C.c_int32 * 3)(*[int(x) for x in (M if hasattr(M, "__len__") else (M,) * 3)])
    m = Mesh()
    _check("hpf_mesh_make", lib().hpf_mesh_make(Lf, Mi, int(n_beads), C.byref(m)))
    return m


def make_field(K: int, kT: float, inv_kappa: float, chi) -> Field:
    f = Field()
    f.K = int(K)
    f.kT = float(kT)
    f.inv_kappa = float(inv_kappa)
    flat = [float(chi[a][b]) for a in range(K) for b in range(K)]
    for i, v in enumerate(flat):
        f.chi[i] = v
    return f


def _nm(mesh: Mesh) -> int:
    return mesh.M[0] * mesh.M[1] * mesh.M[2]


def _box(mesh_or_box):
    if isinstance(mesh_or_box, Mesh):
        return (C.c_float * 3)(*mesh_or_box.L)
    v = [float(x) for x in (mesh_or_box if hasattr(mesh_or_box, "__len__") else (mesh_or_box,) * 3)]
    return (C.c_float * 3)(*v)


def hpf_density_scatter(R, T, mesh: Mesh, K: int, counts, stream=None):
    N = R.shape[0]
    r = _dev(R, "R", torch.float32, (N, 3))
    t = _dev(T, "T", torch.uint8, (N,))
    c = _dev(counts, "counts", _U64, (K, _nm(mesh)))
    _check("hpf_density_scatter",
           lib().hpf_density_scatter(r, t, N, C.byref(mesh), K, c, _stream(stream)))


def hpf_scatter_workspace_bytes(N: int, mesh: Mesh, K: int, B: int = 8, halo: int = 1) -> int:
    """Workspace of hpf_density_scatter_cells; 0 when the sizes are not supported."""
    return int(lib().hpf_scatter_workspace_bytes(int(N), C.byref(mesh), int(K), int(B), int(halo)))


def hpf_density_scatter_cells(R, T, mesh: Mesh, K: int, cell_start, B: int, halo: int, counts, work,
                              stream=None):
    N = R.shape[0]
    r = _dev(R, "R", torch.float32, (N, 3))
    t = _dev(T, "T", torch.uint8, (N,))
    cs = _dev(cell_start, "cell_start", torch.int32, (sort_key_count(mesh, B) + 2,))
    c = _dev(counts, "counts", _U64, (K, _nm(mesh)))
    w = _dev(work, "work", (torch.uint8, torch.int32))
    _check("hpf_density_scatter_cells",
           lib().hpf_density_scatter_cells(r, t, N, C.byref(mesh), K, cs, int(B), int(halo), c, w,
                                           work.numel() * work.element_size(), _stream(stream)))


def hpf_density_scatter_cells_static(R, T, mesh: Mesh, K: int, cell_start, B: int, halo: int, counts,
                                     stream=None):
    N = R.shape[0]
    r = _dev(R, "R", torch.float32, (N, 3))
    t = _dev(T, "T", torch.uint8, (N,))
    cs = _dev(cell_start, "cell_start", torch.int32, (sort_key_count(mesh, B) + 2,))
    c = _dev(counts, "counts", _U64, (K, _nm(mesh)))
    _check("hpf_density_scatter_cells_static",
           lib().hpf_density_scatter_cells_static(r, t, N, C.byref(mesh), K, cs, int(B), int(halo), c,
                                                  _stream(stream)))


def hpf_field_potential(counts, mesh: Mesh, field: Field, V, w_part=None, stream=None, present=None):
    nm, K = _nm(mesh), field.K
    c = _dev(counts, "counts", _U64, (K, nm))
    v = _dev(V, "V", torch.float32, (K, nm))
    w = _dev(w_part, "w_part", torch.float64, None, allow_none=True)
    if w_part is not None and w_part.numel() < HPF_NPART:
        raise ValueError("w_part needs HPF_NPART slots")
    _check("hpf_field_potential",
           lib().hpf_field_potential(c, C.byref(mesh), C.byref(field), v, w,
                                     _dev(present, "present", torch.uint8, (nm,), allow_none=True),
                                     _stream(stream)))


def hpf_field_gradient(V, mesh: Mesh, K: int, G, stream=None, present=None):
    nm = _nm(mesh)
    v = _dev(V, "V", torch.float32, (K, nm))
    g = _dev(G, "G", torch.float32, (K, nm, 3))
    pr = _dev(present, "present", torch.uint8, (nm,), allow_none=True)
    _check("hpf_field_gradient", lib().hpf_field_gradient(v, C.byref(mesh), K, g, pr, _stream(stream)))


def hpf_force_gather(R, T, mesh: Mesh, K: int, G, F, stream=None):
    N, nm = R.shape[0], _nm(mesh)
    r = _dev(R, "R", torch.float32, (N, 3))
    t = _dev(T, "T", torch.uint8, (N,))
    g = _dev(G, "G", torch.float32, (K, nm, 3))
    f = _dev(F, "F", torch.float32, (N, 3))
    _check("hpf_force_gather",
           lib().hpf_force_gather(r, t, N, C.byref(mesh), K, g, f, _stream(stream)))


def hpf_force_gather_staggered(R, T, mesh: Mesh, K: int, V, F, stream=None):
    N = R.shape[0]
    _check("hpf_force_gather_staggered", lib().hpf_force_gather_staggered(
        _dev(R, "R", torch.float32, (N, 3)), _dev(T, "T", torch.uint8, (N,)), N, C.byref(mesh), int(K),
        _dev(V, "V", torch.float32, (K, _nm(mesh))), _dev(F, "F", torch.float32, (N, 3)),
        _stream(stream)))


def bond_forces(R, bonds, k: float, r0: float, box, F, e_part=None, stream=None):
    N = R.shape[0]
    D = bonds.shape[0] if bonds is not None else 0
    r = _dev(R, "R", torch.float32, (N, 3))
    b = _dev(bonds, "bonds", torch.int32, (D, N), allow_none=True) if D else None
    f = _dev(F, "F", torch.float32, (N, 3))
    e = _dev(e_part, "e_part", torch.float64, None, allow_none=True)
    if e_part is not None and e_part.numel() < HPF_NPART:
        raise ValueError("e_part needs HPF_NPART slots")
    _check("bond_forces", lib().bond_forces(r, N, b, D, float(k), float(r0), _box(box), f, e,
                                            _stream(stream)))


def angle_forces(R, angles, k, theta0, form, box, F, e_part=None, stream=None):
    """Angle forces (Bonded forces section) added to F; angles is the per-bead table [3A, N]
    (None = no angles); k, theta0 (radians), form: one value per angle type."""
    N = R.shape[0]
    A = angles.shape[0] // 3 if angles is not None else 0
    kk = [float(x) for x in (k if hasattr(k, "__len__") else (k,))]
    nt = len(kk)
    th = [float(x) for x in (theta0 if hasattr(theta0, "__len__") else (theta0,) * nt)]
    fm = [int(x) for x in (form if hasattr(form, "__len__") else (form,) * nt)]
    if e_part is not None and e_part.numel() < HPF_NPART:
        raise ValueError("e_part needs HPF_NPART slots")
    _check("angle_forces", lib().angle_forces(
        _dev(R, "R", torch.float32, (N, 3)), N,
        _dev(angles, "angles", torch.int32, (3 * A, N), allow_none=True) if A else None, A, nt,
        (C.c_float * nt)(*kk), (C.c_float * nt)(*th), (C.c_int32 * nt)(*fm), _box(box),
        _dev(F, "F", torch.float32, (N, 3)),
        _dev(e_part, "e_part", torch.float64, None, allow_none=True), _stream(stream)))


def hpf_sort_angles(mesh: Mesh, B: int, angles_in, angles_out, work, stream=None):
    N = angles_in.shape[1]
    A = angles_in.shape[0] // 3
    _check("hpf_sort_angles", lib().hpf_sort_angles(
        C.byref(mesh), int(B), N, _dev(angles_in, "angles_in", torch.int32, (3 * A, N)), A,
        _dev(angles_out, "angles_out", torch.int32, (3 * A, N)), _dev(work, "work", torch.uint8),
        work.numel(), _stream(stream)))


def verlet_step(R, Vel, F, dt: float, box, half: int, inv_mass=None, kin_part=None, stream=None):
    N = Vel.shape[0]
    r = _dev(R, "R", torch.float32, (N, 3), allow_none=(half == 2))
    v = _dev(Vel, "Vel", torch.float32, (N, 3))
    f = _dev(F, "F", torch.float32, (N, 3))
    im = _dev(inv_mass, "inv_mass", torch.float32, (N,), allow_none=True)
    kp = _dev(kin_part, "kin_part", torch.float64, None, allow_none=True)
    if kin_part is not None and kin_part.numel() < 4 * HPF_NPART:
        raise ValueError("kin_part needs 4 * HPF_NPART slots")
    _check("verlet_step", lib().verlet_step(r, v, f, im, N, float(dt), _box(box), int(half), kp,
                                            _stream(stream)))


def hpf_advance(R, R_next, Vel, T, mesh: Mesh, K: int, G, bonds, k: float, r0: float, box,
                dt: float, inv_mass=None, F_out=None, e_part=None, kin_part=None, thermostat=None,
                stream=None):
    N = R.shape[0]
    D = bonds.shape[0] if bonds is not None else 0
    args = [
        _dev(R, "R", torch.float32, (N, 3)),
        _dev(R_next, "R_next", torch.float32, (N, 3)),
        _dev(Vel, "Vel", torch.float32, (N, 3)),
        _dev(T, "T", torch.uint8, (N,)),
        N, C.byref(mesh), int(K),
        _dev(G, "G", torch.float32, (K, _nm(mesh), 3)),
        _dev(bonds, "bonds", torch.int32, (D, N), allow_none=True) if D else None,
        int(D), float(k), float(r0), _box(box),
        _dev(inv_mass, "inv_mass", torch.float32, (N,), allow_none=True),
        float(dt),
        _dev(F_out, "F_out", torch.float32, (N, 3), allow_none=True),
        _dev(e_part, "e_part", torch.float64, None, allow_none=True),
        _dev(kin_part, "kin_part", torch.float64, None, allow_none=True),
    ]
    if e_part is not None and e_part.numel() < HPF_NPART:
        raise ValueError("e_part needs HPF_NPART slots")
    if kin_part is not None and kin_part.numel() < 4 * HPF_NPART:
        raise ValueError("kin_part needs 4 * HPF_NPART slots")
    _check("hpf_advance", lib().hpf_advance(*args, _thermo(thermostat), _stream(stream)))


def _thermo(th):
    return None if th is None else C.byref(th)


def hpf_andersen(Vel, thermostat: Thermostat, inv_mass=None, kin_part=None, stream=None):
    N = Vel.shape[0]
    if kin_part is not None and kin_part.numel() < 4 * HPF_NPART:
        raise ValueError("kin_part needs 4 * HPF_NPART slots")
    _check("hpf_andersen", lib().hpf_andersen(
        _dev(Vel, "Vel", torch.float32, (N, 3)),
        _dev(inv_mass, "inv_mass", torch.float32, (N,), allow_none=True), N, C.byref(thermostat),
        _dev(kin_part, "kin_part", torch.float64, None, allow_none=True), _stream(stream)))


def hpf_advance_scatter(R, R_next, Vel, T, mesh: Mesh, K: int, G, bonds, k: float, r0: float, box,
                        dt: float, cell_start, B: int, halo: int, counts, work, inv_mass=None,
                        F_out=None, e_part=None, kin_part=None, thermostat=None, stream=None):
    N = R.shape[0]
    D = bonds.shape[0] if bonds is not None else 0
    args = [
        _dev(R, "R", torch.float32, (N, 3)),
        _dev(R_next, "R_next", torch.float32, (N, 3)),
        _dev(Vel, "Vel", torch.float32, (N, 3)),
        _dev(T, "T", torch.uint8, (N,)),
        N, C.byref(mesh), int(K),
        _dev(G, "G", torch.float32, (K, _nm(mesh), 3)),
        _dev(bonds, "bonds", torch.int32, (D, N), allow_none=True) if D else None,
        int(D), float(k), float(r0), _box(box),
        _dev(inv_mass, "inv_mass", torch.float32, (N,), allow_none=True),
        float(dt),
        _dev(cell_start, "cell_start", torch.int32, (sort_key_count(mesh, B) + 2,)),
        int(B), int(halo),
        _dev(counts, "counts", torch.int64, (K, _nm(mesh))),
        _dev(work, "work", torch.uint8), work.numel(),
        _dev(F_out, "F_out", torch.float32, (N, 3), allow_none=True),
        _dev(e_part, "e_part", torch.float64, None, allow_none=True),
        _dev(kin_part, "kin_part", torch.float64, None, allow_none=True),
    ]
    if e_part is not None and e_part.numel() < HPF_NPART:
        raise ValueError("e_part needs HPF_NPART slots")
    if kin_part is not None and kin_part.numel() < 4 * HPF_NPART:
        raise ValueError("kin_part needs 4 * HPF_NPART slots")
    _check("hpf_advance_scatter", lib().hpf_advance_scatter(*args, _thermo(thermostat),
                                                            _stream(stream)))


def hpf_density_finish_cells(counts, N: int, mesh: Mesh, K: int, B: int, halo: int, work,
                             stream=None):
    c = _dev(counts, "counts", torch.int64, (K, _nm(mesh)))
    w = _dev(work, "work", torch.uint8)
    _check("hpf_density_finish_cells",
           lib().hpf_density_finish_cells(c, int(N), C.byref(mesh), int(K), int(B), int(halo), w,
                                          work.numel(), _stream(stream)))


def hpf_field_potential_cells(counts, N: int, mesh: Mesh, field: Field, B: int, halo: int, work, V,
                              w_part=None, stream=None, present=None):
    K = field.K
    c = _dev(counts, "counts", torch.int64, (K, _nm(mesh)))
    w = _dev(work, "work", torch.uint8)
    v = _dev(V, "V", torch.float32, (K, _nm(mesh)))
    wp = _dev(w_part, "w_part", torch.float64, None, allow_none=True)
    if w_part is not None and w_part.numel() < HPF_NPART:
        raise ValueError("w_part needs HPF_NPART slots")
    _check("hpf_field_potential_cells",
           lib().hpf_field_potential_cells(c, int(N), C.byref(mesh), C.byref(field), int(B), int(halo), w,
                                           work.numel(), v, wp,
                                           _dev(present, "present", torch.uint8, (_nm(mesh),),
                                                allow_none=True), _stream(stream)))


def hpf_reduce_partials(part, ncomp: int, out, stream=None):
    p = _dev(part, "part", torch.float64)
    o = _dev(out, "out", torch.float64)
    if part.numel() < ncomp * HPF_NPART or out.numel() < ncomp:
        raise ValueError("partial buffer or output too small")
    _check("hpf_reduce_partials", lib().hpf_reduce_partials(p, int(ncomp), o, _stream(stream)))


def hpf_sort_workspace_bytes(N: int, mesh: Mesh, B: int = 8) -> int:
    n = lib().hpf_sort_workspace_bytes(int(N), C.byref(mesh), int(B))
    if n == 0:
        raise HpfError("hpf_sort_workspace_bytes", -1, "invalid mesh, size or brick")
    return int(n)


def sort_key_count(mesh: Mesh, B: int = 8) -> int:
    """NK: number of sort keys, one per brick of B^3 cells (cell_start needs NK + 2)."""
    B = B or 8
    n = 1
    for d in range(3):
        n *= (mesh.M[d] + B - 1) // B
    return n


def hpf_resort_by_cell(mesh: Mesh, B: int, R_in, Vel_in, T_in, tag_in, bonds_in, R_out, Vel_out,
                       T_out, tag_out, bonds_out, work, cell_start_in, cell_start_out, stream=None):
    N = R_in.shape[0]
    D = bonds_in.shape[0] if bonds_in is not None else 0
    nk = sort_key_count(mesh, B)
    args = [
        _dev(R_in, "R_in", torch.float32, (N, 3)),
        _dev(Vel_in, "Vel_in", torch.float32, (N, 3), allow_none=True),
        _dev(T_in, "T_in", torch.uint8, (N,)),
        _dev(tag_in, "tag_in", torch.int32, (N,), allow_none=True),
        _dev(bonds_in, "bonds_in", torch.int32, (D, N), allow_none=True) if D else None,
        int(D),
        _dev(R_out, "R_out", torch.float32, (N, 3)),
        _dev(Vel_out, "Vel_out", torch.float32, (N, 3), allow_none=True),
        _dev(T_out, "T_out", torch.uint8, (N,)),
        _dev(tag_out, "tag_out", torch.int32, (N,), allow_none=True),
        _dev(bonds_out, "bonds_out", torch.int32, (D, N), allow_none=True) if D else None,
        _dev(cell_start_in, "cell_start_in", torch.int32, (nk + 2,)),
        _dev(cell_start_out, "cell_start_out", torch.int32, (nk + 2,)),
    ]
    w = _dev(work, "work", torch.uint8)
    _check("hpf_resort_by_cell",
           lib().hpf_resort_by_cell(C.byref(mesh), int(B), N, *args, w, work.numel(), _stream(stream)))


def hpf_sort_by_cell(mesh: Mesh, B: int, R_in, Vel_in, T_in, tag_in, bonds_in, R_out, Vel_out,
                     T_out, tag_out, bonds_out, work, cell_start=None, stream=None):
    N = R_in.shape[0]
    D = bonds_in.shape[0] if bonds_in is not None else 0
    args = [
        _dev(R_in, "R_in", torch.float32, (N, 3)),
        _dev(Vel_in, "Vel_in", torch.float32, (N, 3), allow_none=True),
        _dev(T_in, "T_in", torch.uint8, (N,)),
        _dev(tag_in, "tag_in", torch.int32, (N,), allow_none=True),
        _dev(bonds_in, "bonds_in", torch.int32, (D, N), allow_none=True) if D else None,
        int(D),
        _dev(R_out, "R_out", torch.float32, (N, 3)),
        _dev(Vel_out, "Vel_out", torch.float32, (N, 3), allow_none=True),
        _dev(T_out, "T_out", torch.uint8, (N,)),
        _dev(tag_out, "tag_out", torch.int32, (N,), allow_none=True),
        _dev(bonds_out, "bonds_out", torch.int32, (D, N), allow_none=True) if D else None,
    ]
    cs = None
    if cell_start is not None:
        nk = sort_key_count(mesh, B)
        cs = _dev(cell_start, "cell_start", torch.int32, (nk + 2,))
    w = _dev(work, "work", torch.uint8)
    _check("hpf_sort_by_cell",
           lib().hpf_sort_by_cell(C.byref(mesh), int(B), N, *args, cs, w, work.numel(),
                                  _stream(stream)))


def hpf_get_device_status(clear: bool = True, stream=None) -> int:
    flags = C.c_uint32(0)
    _check("hpf_get_device_status",
           lib().hpf_get_device_status(C.byref(flags), int(bool(clear)), _stream(stream)))
    return int(flags.value)


# ------------------------------------------------------------ batch / graph

def hpf_batch_workspace_bytes(reps, cfg: BatchConfig) -> int:
    arr = (Replica * len(reps))(*reps)
    return int(lib().hpf_batch_workspace_bytes(arr, len(reps), C.byref(cfg)))


def hpf_batch_create(reps, cfg: BatchConfig, bufs: BatchBuffers, work) -> C.c_void_p:
    arr = (Replica * len(reps))(*reps)
    h = C.c_void_p()
    w = _dev(work, "work", torch.uint8)
    _check("hpf_batch_create", lib().hpf_batch_create(arr, len(reps), C.byref(cfg), C.byref(bufs), w,
                                                      work.numel(), C.byref(h)))
    return h


def hpf_batch_start(h, stream=None):
    _check("hpf_batch_start", lib().hpf_batch_start(h, _stream(stream)))


def hpf_batch_step(h, n_steps: int, report_last: bool = True, stream=None):
    _check("hpf_batch_step", lib().hpf_batch_step(h, int(n_steps), int(bool(report_last)),
                                                  _stream(stream)))


def hpf_batch_current(h) -> dict:
    ptrs = [C.c_void_p() for _ in range(6)]
    _check("hpf_batch_current", lib().hpf_batch_current(h, *[C.byref(p) for p in ptrs]))
    return dict(zip(["R", "Vel", "T", "tag", "bonds", "energies"], [p.value for p in ptrs]))


def hpf_batch_density(h, counts_out, stream=None):
    _check("hpf_batch_density", lib().hpf_batch_density(h, _dev(counts_out, "counts_out", _U64),
                                                        _stream(stream)))


def hpf_batch_tune(h, trial_steps: int, stream=None):
    cfg = BatchConfig()
    ms = (C.c_float * 32)()
    n = C.c_int32()
    _check("hpf_batch_tune", lib().hpf_batch_tune(h, int(trial_steps), _stream(stream),
                                                  C.byref(cfg), ms, C.byref(n)))
    return cfg, [ms[i] for i in range(n.value)]


def hpf_batch_destroy(h):
    _check("hpf_batch_destroy", lib().hpf_batch_destroy(h))


def hpf_graph_begin(stream):
    _check("hpf_graph_begin", lib().hpf_graph_begin(_stream(stream)))


def hpf_graph_end(stream) -> C.c_void_p:
    g = C.c_void_p()
    _check("hpf_graph_end", lib().hpf_graph_end(_stream(stream), C.byref(g)))
    return g


def hpf_graph_launch(g, stream=None):
    _check("hpf_graph_launch", lib().hpf_graph_launch(g, _stream(stream)))


def hpf_graph_destroy(g):
    _check("hpf_graph_destroy", lib().hpf_graph_destroy(g))
