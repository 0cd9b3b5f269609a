"""Python access to the FP64 CPU oracle (``hpf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the package smoke
check and by the benchmark's CPU-baseline leg. The product path (the HIP
library and its binding) never imports this package.

Arrays follow the oracle's own layout: positions and forces are float64
[N, 3]; meshes are [K, Mz, My, Mx] (x fastest); gradients carry a trailing
axis of 3. FP32 inputs (the [N, 4] bead arrays of the workloads) are widened
to double, which is exact.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hpf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra", "-Wno-unknown-pragmas"]
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "hpf_oracle.h"))):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def build_omp(force: bool = True) -> str:
    """The same source compiled with OpenMP into ``oracle/liboracle_omp.so``: used only to
    time the oracle on all host cores (FP64 sums regrouped by thread; counts still exact)."""
    if not force and os.path.exists(_LIB_OMP) and os.path.getmtime(_LIB_OMP) >= max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "hpf_oracle.h"))):
        return _LIB_OMP
    tmp = _LIB_OMP + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", *CFLAGS, "-fopenmp", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_OMP)
    return _LIB_OMP


class _Mesh(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("M", C.c_int32 * 3), ("s", C.c_float * 3)]


class _Params(C.Structure):
    _fields_ = [("mesh", C.POINTER(_Mesh)), ("K", C.c_int32), ("kT", C.c_double),
                ("inv_kappa", C.c_double), ("chi", C.POINTER(C.c_double)),
                ("bonds", C.POINTER(C.c_int32)), ("D", C.c_int32), ("k_bond", C.c_double),
                ("r0", C.c_double)]


_lib = None
_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        _lib = _declare(C.CDLL(build(force=False)))
    return _lib


def lib_omp(threads: int):
    """The OpenMP build (timing only), set to `threads` threads."""
    global _lib_omp
    if _lib_omp is None:
        _lib_omp = _declare(C.CDLL(build_omp(force=False)))
        _lib_omp.omp_set_num_threads.argtypes = [C.c_int]
    _lib_omp.omp_set_num_threads(int(threads))
    return _lib_omp


def _declare(_lib):
    if True:
        P = C.c_void_p
        _lib.or_mesh_init.argtypes = [C.POINTER(_Mesh), P, P]
        _lib.or_cell_weights.argtypes = [C.c_double, C.c_float, C.c_int32,
                                         C.POINTER(C.c_int32), P]
        _lib.or_cell_weights.restype = C.c_int
        _lib.or_density.argtypes = [P, P, C.c_int64, C.POINTER(_Mesh), C.c_int32, P]
        _lib.or_density.restype = C.c_int64
        _lib.or_potential.argtypes = [P, C.POINTER(_Mesh), C.c_int64, C.c_int32, C.c_double,
                                      C.c_double, P, P, P]
        _lib.or_gradient.argtypes = [P, C.POINTER(_Mesh), C.c_int32, P]
        _lib.or_gather.argtypes = [P, P, C.c_int64, C.POINTER(_Mesh), C.c_int32, P, P]
        _lib.or_gather.restype = C.c_int64
        _lib.or_bonds.argtypes = [P, C.c_int64, P, C.c_int32, C.c_double, C.c_double, P, P, P]
        _lib.or_verlet_half1.argtypes = [P, P, P, P, C.c_int64, C.c_double, P]
        _lib.or_verlet_half2.argtypes = [P, P, P, C.c_int64, C.c_double, P]
        _lib.or_forces.argtypes = [P, P, C.c_int64, C.POINTER(_Params), P, P, P]
        _lib.or_forces.restype = C.c_int64
        _lib.or_run.argtypes = [P, P, P, P, C.c_int64, C.POINTER(_Params), C.c_double,
                                C.c_int32, P]
        _lib.or_run.restype = C.c_int
        _lib.or_run_interval.argtypes = [P, P, P, P, C.c_int64, C.POINTER(_Params), C.c_double,
                                         C.c_int32, C.c_int32, P]
        _lib.or_run_interval.restype = C.c_int
        _lib.or_sort_perm.argtypes = [P, P, C.c_int64, C.POINTER(_Mesh), C.c_int32, P, P]
        _lib.or_sort_perm.restype = C.c_int
        _lib.or_gather_staggered.argtypes = [P, P, C.c_int64, C.POINTER(_Mesh), C.c_int32, P, P, P]
        _lib.or_gather_staggered.restype = C.c_int64
        _lib.or_angles.argtypes = [P, C.c_int64, P, C.c_int32, C.c_int32, P, P, P, P, P, P]
        _lib.or_philox4x32_10.argtypes = [P, P, P]
        _lib.or_andersen.argtypes = [P, P, P, C.c_int64, C.c_double, C.c_float, C.c_uint64,
                                     C.c_int64, P]
        _lib.or_andersen.restype = C.c_int64
        _lib.or_run_nvt.argtypes = [P, P, P, P, P, C.c_int64, C.POINTER(_Params), C.c_double,
                                    C.c_int32, C.c_int32, C.c_double, C.c_float, C.c_uint64, P]
        _lib.or_run_nvt.restype = C.c_int
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def mesh(L, M) -> _Mesh:
    Lf = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float32), (3,)))
    Mi = np.ascontiguousarray(np.broadcast_to(np.asarray(M, dtype=np.int32), (3,)))
    m = _Mesh()
    lib().or_mesh_init(C.byref(m), _p(Lf), _p(Mi))
    return m


def _pos(R) -> np.ndarray:
    R = np.asarray(R)
    if R.dtype == np.float64 and R.ndim == 2 and R.shape[1] == 3:
        return np.ascontiguousarray(R)
    return np.ascontiguousarray(R[:, :3], dtype=np.float64)


def _box(L) -> np.ndarray:
    return np.ascontiguousarray(
        np.broadcast_to(np.asarray(L, dtype=np.float32), (3,)).astype(np.float64))


def cell_weights(x: float, s, M: int):
    c = C.c_int32()
    w = np.zeros(2, dtype=np.uint32)
    bad = lib().or_cell_weights(float(x), C.c_float(float(s)), int(M), C.byref(c), _p(w))
    return bad, c.value, w


def density(R, T, L, M, K):
    m = mesh(L, M)
    Rd = _pos(R)
    T = np.ascontiguousarray(T, dtype=np.uint8)
    counts = np.zeros((K, m.M[2], m.M[1], m.M[0]), dtype=np.uint64)
    skipped = lib().or_density(_p(Rd), _p(T), len(T), C.byref(m), K, _p(counts))
    return counts, int(skipped)


def potential(counts, L, M, n_beads, kT, inv_kappa, chi):
    m = mesh(L, M)
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    K = counts.shape[0]
    chi = np.ascontiguousarray(chi, dtype=np.float64).reshape(K, K)
    V = np.zeros(counts.shape, dtype=np.float64)
    W = C.c_double()
    lib().or_potential(_p(counts), C.byref(m), int(n_beads), K, float(kT), float(inv_kappa),
                       _p(chi), _p(V), C.byref(W))
    return V, W.value


def gradient(V, L, M):
    m = mesh(L, M)
    V = np.ascontiguousarray(V, dtype=np.float64)
    G = np.zeros(V.shape + (3,), dtype=np.float64)
    lib().or_gradient(_p(V), C.byref(m), V.shape[0], _p(G))
    return G


def gather(R, T, L, M, G):
    m = mesh(L, M)
    Rd = _pos(R)
    T = np.ascontiguousarray(T, dtype=np.uint8)
    G = np.ascontiguousarray(G, dtype=np.float64)
    F = np.zeros((len(T), 3), dtype=np.float64)
    lib().or_gather(_p(Rd), _p(T), len(T), C.byref(m), G.shape[0], _p(G), _p(F))
    return F


def bonds(R, bond_table, k, r0, L):
    Rd = _pos(R)
    b = np.ascontiguousarray(bond_table, dtype=np.int32)
    N = Rd.shape[0]
    F = np.zeros((N, 3), dtype=np.float64)
    E = C.c_double()
    lib().or_bonds(_p(Rd), N, _p(b), b.shape[0] if N else 0, float(k), float(r0), _p(_box(L)),
                   _p(F), C.byref(E))
    return F, E.value


def verlet_half1(R, V, F, dt, L, inv_mass=None):
    R = _pos(R).copy()
    V = _pos(V).copy()
    F = np.ascontiguousarray(F, dtype=np.float64)
    im = None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64)
    lib().or_verlet_half1(_p(R), _p(V), _p(F), None if im is None else _p(im), R.shape[0],
                          float(dt), _p(_box(L)))
    return R, V


def verlet_half2(V, F, dt, inv_mass=None):
    V = _pos(V).copy()
    F = np.ascontiguousarray(F, dtype=np.float64)
    im = None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64)
    out = np.zeros(4)
    lib().or_verlet_half2(_p(V), _p(F), None if im is None else _p(im), V.shape[0], float(dt),
                          _p(out))
    return V, out


def _params(m, sys_like, chi, bond_table, keep):
    K = int(sys_like["K"])
    chi = np.ascontiguousarray(chi, dtype=np.float64).reshape(K, K)
    b = np.ascontiguousarray(bond_table, dtype=np.int32)
    keep += [chi, b]
    p = _Params()
    p.mesh = C.pointer(m)
    p.K = K
    p.kT = float(sys_like["kT"])
    p.inv_kappa = float(sys_like["inv_kappa"])
    p.chi = chi.ctypes.data_as(C.POINTER(C.c_double))
    p.bonds = b.ctypes.data_as(C.POINTER(C.c_int32))
    p.D = b.shape[0]
    p.k_bond = float(sys_like["k_bond"])
    p.r0 = float(sys_like["r0"])
    return p


def _sysdict(s):
    return {"K": s.K, "kT": s.kT, "inv_kappa": s.inv_kappa, "k_bond": s.k_bond, "r0": s.r0}


def forces(sys, R=None):
    """Field and bond forces of a ``synth.workloads.System`` (positions R if given)."""
    m = mesh(sys.L, sys.M)
    keep = []
    p = _params(m, _sysdict(sys), sys.chi, sys.bonds, keep)
    Rd = _pos(sys.R if R is None else R)
    T = np.ascontiguousarray(sys.T, dtype=np.uint8)
    N = Rd.shape[0]
    Ff = np.zeros((N, 3))
    Fb = np.zeros((N, 3))
    e2 = np.zeros(2)
    rc = lib().or_forces(_p(Rd), _p(T), N, C.byref(p), _p(Ff), _p(Fb), _p(e2))
    if rc < 0:
        raise MemoryError("oracle allocation failed")
    return Ff, Fb, {"W": e2[0], "E_bond": e2[1], "skipped": int(rc)}


def run(sys, n_steps, R=None, V=None, inv_mass=None, threads=None):
    """Velocity Verlet for n_steps; returns (R, V, energies[n_steps+1, 4] = KE, Eb, W, Etot).
    With `threads`, the OpenMP build runs it on that many host threads (timing only: its FP64
    sums are regrouped, so the energies may differ in the last bits)."""
    m = mesh(sys.L, sys.M)
    keep = []
    p = _params(m, _sysdict(sys), sys.chi, sys.bonds, keep)
    Rd = _pos(sys.R if R is None else R).copy()
    Vd = _pos(sys.V if V is None else V).copy()
    T = np.ascontiguousarray(sys.T, dtype=np.uint8)
    im = None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64)
    E = np.zeros((n_steps + 1, 4))
    L = lib() if threads is None else lib_omp(threads)
    rc = L.or_run(_p(Rd), _p(Vd), _p(T), None if im is None else _p(im), Rd.shape[0],
                  C.byref(p), float(sys.dt), int(n_steps), _p(E))
    if rc:
        raise MemoryError("oracle allocation failed")
    return Rd, Vd, E


def run_interval(sys, n_steps, field_every, R=None, V=None, inv_mass=None):
    """run() with the density field rebuilt only every `field_every` force evaluations
    (O11: the MD-SCF section's field-update interval); field_every = 1 is run()."""
    m = mesh(sys.L, sys.M)
    keep = []
    p = _params(m, _sysdict(sys), sys.chi, sys.bonds, keep)
    Rd = _pos(sys.R if R is None else R).copy()
    Vd = _pos(sys.V if V is None else V).copy()
    T = np.ascontiguousarray(sys.T, dtype=np.uint8)
    im = None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64)
    E = np.zeros((n_steps + 1, 4))
    rc = lib().or_run_interval(_p(Rd), _p(Vd), _p(T), None if im is None else _p(im), Rd.shape[0],
                               C.byref(p), float(sys.dt), int(n_steps), int(field_every), _p(E))
    if rc == -2:
        raise ValueError("field_every must be >= 1")
    if rc:
        raise MemoryError("oracle allocation failed")
    return Rd, Vd, E


def sort_perm(R, tag, L, M, B):
    m = mesh(L, M)
    Rd = _pos(R)
    tag = np.ascontiguousarray(tag, dtype=np.int32)
    N = Rd.shape[0]
    perm = np.zeros(N, dtype=np.int64)
    keys = np.zeros(N, dtype=np.uint32)
    if lib().or_sort_perm(_p(Rd), _p(tag), N, C.byref(m), int(B), _p(perm), _p(keys)):
        raise MemoryError("oracle allocation failed")
    return perm, keys


def philox4x32_10(ctr, key):
    """O12: the four 32-bit outputs of Philox4x32-10 for a counter (4 words) and key (2)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def andersen(V, tag, kT, p, seed, step, inv_mass=None):
    """O13: velocities after the Andersen collisions of time level `step`; returns
    (V [N, 3] float64, collision mask uint8 [N])."""
    Vd = _pos(V).copy()
    tg = np.ascontiguousarray(tag, dtype=np.int32)
    im = None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64)
    mask = np.zeros(Vd.shape[0], dtype=np.uint8)
    lib().or_andersen(_p(Vd), _p(tg), None if im is None else _p(im), Vd.shape[0], float(kT),
                      float(p), int(seed), int(step), _p(mask))
    return Vd, mask


def run_nvt(sys, n_steps, field_every, kT, p, seed, R=None, V=None, inv_mass=None):
    """run_interval() with the Andersen thermostat after the second half kick of every step
    (O13); p = collision probability per step. Returns (R, V, energies[n_steps+1, 4])."""
    m = mesh(sys.L, sys.M)
    keep = []
    prm = _params(m, _sysdict(sys), sys.chi, sys.bonds, keep)
    Rd = _pos(sys.R if R is None else R).copy()
    Vd = _pos(sys.V if V is None else V).copy()
    T = np.ascontiguousarray(sys.T, dtype=np.uint8)
    tg = np.ascontiguousarray(sys.tag, dtype=np.int32)
    im = None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64)
    E = np.zeros((n_steps + 1, 4))
    rc = lib().or_run_nvt(_p(Rd), _p(Vd), _p(T), _p(tg), None if im is None else _p(im), Rd.shape[0],
                          C.byref(prm), float(sys.dt), int(n_steps), int(field_every), float(kT),
                          float(p), int(seed), _p(E))
    if rc:
        raise MemoryError("oracle allocation failed")
    return Rd, Vd, E


def gather_staggered(R, T, L, M, Phi, A):
    """O7P: the staggered nearest-vertex force (reading P of Algorithm 1 Kernels 3-4) of fields
    Phi [K, Mz, My, Mx] with coefficients A [K, K]; returns F [N, 3]."""
    m = mesh(L, M)
    Rd = _pos(R)
    Td = np.ascontiguousarray(T, dtype=np.uint8)
    Pd = np.ascontiguousarray(Phi, dtype=np.float64)
    K = Pd.shape[0]
    Ad = np.ascontiguousarray(A, dtype=np.float64).reshape(K, K)
    F = np.zeros((Rd.shape[0], 3))
    lib().or_gather_staggered(_p(Rd), _p(Td), Rd.shape[0], C.byref(m), K, _p(Pd), _p(Ad), _p(F))
    return F


def angles(R, angle_table, k, theta0, form, L):
    """O8A: angle forces F [N, 3] and energy of a per-bead angle table [3A, N] (rows partner,
    partner, role + 2 type per slot); k, theta0, form are scalars (one type) or per-type
    sequences; form 0 = k (theta - theta0)^2, 1 = k (cos theta - cos theta0)^2."""
    Rd = _pos(R)
    N = Rd.shape[0]
    tab = np.ascontiguousarray(angle_table, dtype=np.int32)
    A = tab.shape[0] // 3 if tab.size else 0
    kk = np.atleast_1d(np.asarray(k, dtype=np.float64)).copy()
    th = np.broadcast_to(np.asarray(theta0, dtype=np.float64), kk.shape).copy()
    fm = np.broadcast_to(np.asarray(form, dtype=np.int32), kk.shape).copy()
    F = np.zeros((N, 3))
    E = C.c_double(0.0)
    lib().or_angles(_p(Rd), N, _p(tab) if A else None, A, kk.size, _p(kk), _p(th), _p(fm),
                    _p(_box(L)), _p(F), C.byref(E))
    return F, E.value
