"""Seeded synthetic hPF-MD systems: bead positions, velocities, types, tags, bond tables.

This module only *draws* inputs. It holds none of the method's arithmetic (no
mesh assignment, no potential, no forces, no integration), so both the FP64
oracle and the HIP path can take their inputs from it without sharing any part
of the computation.

The systems stand in for the paper's coarse-grained polymer workloads (the
lipid/water MD-SCF benchmark of the performance section, whose force-field
parameters are not available): linear bead-spring chains drawn as random walks
of fixed step length in a cubic periodic box at bead density about 3, with the
chain architectures, Flory-Huggins parameters, compressibility and mesh sizes
of the five named workloads below.

Recipe (all workloads):
  * numpy PCG64 generator seeded with ``13102041 + index``;
  * every chain starts at a uniform random point of the box and grows as a
    random walk whose steps have length ``bond_len`` (0.97) and directions
    uniform on the sphere (normalised 3-D normals); positions are then wrapped
    into [0, L) (a coordinate that rounds to L in FP32 is set to 0);
  * velocities are N(0, 1) per component (Maxwell at kT = 1, unit mass) with
    the centre-of-mass velocity subtracted;
  * free solvent beads (the three-species workload) sit at uniform positions;
  * the bond table is the paper's table form (bonded partners of bead i at
    ``bonds[k*N + i]``), here with k in {0, 1} = previous / next bead of the
    chain and -1 for "no partner";
  * types: 0 = A, 1 = B, 2 = W.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 13102041


@dataclass
class System:
    name: str
    R: np.ndarray          # float32 [N, 3]  (x, y, z)
    V: np.ndarray          # float32 [N, 3]  (vx, vy, vz)
    T: np.ndarray          # uint8   [N]
    tag: np.ndarray        # int32   [N]
    bonds: np.ndarray      # int32   [2, N]  (-1 = none)
    L: tuple               # box edges (float)
    M: tuple               # mesh points per edge
    K: int                 # number of species
    kT: float
    inv_kappa: float
    chi: np.ndarray        # float64 [K, K], symmetric
    k_bond: float
    r0: float
    dt: float
    meta: dict = field(default_factory=dict)
    # angle table [3A, N] (partner, partner, role + 2 type per slot) and per-type
    # parameters (k, theta0 in radians, form 0 = harmonic in theta, 1 = in cos theta)
    angles: np.ndarray | None = None
    angle_k: tuple = ()
    angle_theta0: tuple = ()
    angle_form: tuple = ()

    @property
    def N(self) -> int:
        return int(self.R.shape[0])


@dataclass(frozen=True)
class Spec:
    """Parameters of one named workload."""
    name: str
    index: int
    n_chains: int
    chain_len: int
    L: float
    M: int
    K: int
    chi: dict              # {(a, b): value}
    arch: str              # "diblock", "blend", "amphiphile"
    n_block_a: int = 0     # diblock / amphiphile: beads of type A at the chain start
    n_solvent: int = 0
    inv_kappa: float = 10.0
    kT: float = 1.0
    dt: float = 0.03
    k_bond: float = 100.0
    r0: float = 0.0
    bond_len: float = 0.97


# The five workloads. Sizes, box edges, meshes and parameters as named for the
# hPF-MD throughput study; C4 is a batch of replicas (see ``replica_specs``).
SPECS = {
    "c1": Spec("c1_a10b10_diblock_20k", 0, 1000, 20, 18.8, 20, 2, {(0, 1): 1.0},
               "diblock", n_block_a=10),
    "c2": Spec("c2_a20b20_diblock_1m", 1, 25000, 40, 69.3, 64, 2, {(0, 1): 1.5},
               "diblock", n_block_a=20),
    "c3": Spec("c3_ab_blend_10m", 2, 200000, 50, 149.4, 128, 2, {(0, 1): 0.5},
               "blend"),
    # 20 % of 1e8 beads in 12-bead chains is not a whole number of chains:
    # 1,666,667 chains (20,000,004 beads) plus 79,999,996 solvent beads.
    "c5": Spec("c5_amphiphile_solvent_100m", 4, 1666667, 12, 322.0, 256, 3,
               {(0, 1): 1.0, (0, 2): 1.5, (1, 2): -0.5}, "amphiphile",
               n_block_a=4, n_solvent=79999996),
}


def chi_matrix(K: int, chi: dict) -> np.ndarray:
    m = np.zeros((K, K), dtype=np.float64)
    for (a, b), v in chi.items():
        m[a, b] = v
        m[b, a] = v
    return m


def random_walk_chains(rng: np.random.Generator, n_chains: int, chain_len: int,
                       L: float, bond_len: float) -> np.ndarray:
    """Unwrapped float64 positions [n_chains * chain_len, 3] of random-walk chains."""
    start = rng.random((n_chains, 1, 3)) * L
    if chain_len == 1:
        return start.reshape(-1, 3)
    d = rng.standard_normal((n_chains, chain_len - 1, 3))
    d *= bond_len / np.linalg.norm(d, axis=2, keepdims=True)
    pos = np.concatenate([start, start + np.cumsum(d, axis=1)], axis=1)
    return pos.reshape(-1, 3)


def wrap_f32(pos: np.ndarray, L) -> np.ndarray:
    """Wrap float64 positions into [0, L) and round to float32 (L itself maps to 0)."""
    Lv = np.asarray(L, dtype=np.float64)
    w = np.mod(pos, Lv)
    out = w.astype(np.float32)
    Lf = Lv.astype(np.float32)
    out = np.where(out >= Lf, np.float32(0.0), out)
    return out


def maxwell(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    if n:
        v -= v.mean(axis=0, keepdims=True)
    return v


def chain_bonds(n_chains: int, chain_len: int, n_total: int, first: int = 0) -> np.ndarray:
    """Table form bonds [2, n_total]: row 0 = previous bead, row 1 = next bead, -1 = none."""
    b = np.full((2, n_total), -1, dtype=np.int32)
    if chain_len > 1 and n_chains:
        idx = first + np.arange(n_chains * chain_len, dtype=np.int64).reshape(n_chains, chain_len)
        b[0, idx[:, 1:].ravel()] = idx[:, :-1].ravel()
        b[1, idx[:, :-1].ravel()] = idx[:, 1:].ravel()
    return b


def _rows3(xyz: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)


def build(spec: Spec, seed: int | None = None) -> System:
    rng = np.random.default_rng(BASE_SEED + spec.index if seed is None else seed)
    n_chain_beads = spec.n_chains * spec.chain_len
    N = n_chain_beads + spec.n_solvent
    pos = random_walk_chains(rng, spec.n_chains, spec.chain_len, spec.L, spec.bond_len)
    T = np.empty(N, dtype=np.uint8)
    per = np.arange(spec.chain_len)
    if spec.arch in ("diblock", "amphiphile"):
        T[:n_chain_beads] = np.tile(np.where(per < spec.n_block_a, 0, 1), spec.n_chains)
    elif spec.arch == "blend":
        half = spec.n_chains // 2
        T[:half * spec.chain_len] = 0
        T[half * spec.chain_len:n_chain_beads] = 1
    else:
        raise ValueError(spec.arch)
    if spec.n_solvent:
        pos = np.concatenate([pos, rng.random((spec.n_solvent, 3)) * spec.L])
        T[n_chain_beads:] = 2
    R = _rows3(wrap_f32(pos, spec.L))
    V = _rows3(maxwell(rng, N).astype(np.float32))
    bonds = chain_bonds(spec.n_chains, spec.chain_len, N)
    return System(spec.name, R, V, T, np.arange(N, dtype=np.int32), bonds,
                  (spec.L,) * 3, (spec.M,) * 3, spec.K, spec.kT, spec.inv_kappa,
                  chi_matrix(spec.K, spec.chi), spec.k_bond, spec.r0, spec.dt,
                  {"seed": BASE_SEED + spec.index if seed is None else seed,
                   "n_chains": spec.n_chains, "chain_len": spec.chain_len})


def replica_specs(n_rep: int = 64, n_min: int = 8000, n_max: int = 400000,
                  chain_len: int = 20, seed: int = BASE_SEED + 3) -> list:
    """The batched phase-diagram sweep: A10B10 replicas of uneven size.

    Replica 0 has ``n_min`` beads, replica ``n_rep-1`` has ``n_max``; the rest
    are drawn log-uniform between them and rounded to whole chains. The box
    edge is (N_r / 3)^(1/3) (bead density 3), the mesh ceil(L_r) (cell about
    1.0) and chi_AB rises linearly from 0 to 2 across the batch.
    """
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_rep))
    sizes[0], sizes[-1] = n_min, n_max
    out = []
    for r, n in enumerate(sizes):
        nc = max(1, int(round(n / chain_len)))
        L = (nc * chain_len / 3.0) ** (1.0 / 3.0)
        chi_ab = 2.0 * r / (n_rep - 1) if n_rep > 1 else 0.0
        out.append(Spec(f"c4_rep{r:02d}", 3, nc, chain_len, L, int(math.ceil(L)), 2,
                        {(0, 1): chi_ab}, "diblock", n_block_a=chain_len // 2))
    return out


def build_replica(spec: Spec, r: int) -> System:
    return build(spec, seed=BASE_SEED + 3 + 1000 * (r + 1))


def small_system(n_chains: int, chain_len: int, L, M, K: int = 2, seed: int = 7,
                 chi_ab: float = 1.0, n_solvent: int = 0, inv_kappa: float = 10.0) -> System:
    """A small random diblock system with an arbitrary (possibly non-cubic) box.

    Used for ragged sizes, non-cubic meshes and more than two species in the
    parity tests. ``L`` and ``M`` may be scalars or 3-tuples.
    """
    rng = np.random.default_rng(seed)
    Lt = tuple(float(x) for x in (L if np.ndim(L) else (L,) * 3))
    Mt = tuple(int(x) for x in (M if np.ndim(M) else (M,) * 3))
    nb = n_chains * chain_len
    N = nb + n_solvent
    start = rng.random((n_chains, 1, 3)) * np.asarray(Lt)
    if chain_len > 1:
        d = rng.standard_normal((n_chains, chain_len - 1, 3))
        d *= 0.97 / np.linalg.norm(d, axis=2, keepdims=True)
        pos = np.concatenate([start, start + np.cumsum(d, axis=1)], axis=1).reshape(-1, 3)
    else:
        pos = start.reshape(-1, 3)
    if n_solvent:
        pos = np.concatenate([pos, rng.random((n_solvent, 3)) * np.asarray(Lt)])
    T = np.empty(N, dtype=np.uint8)
    T[:nb] = np.tile(np.where(np.arange(chain_len) < chain_len // 2, 0, 1 % K), n_chains)
    if n_solvent:
        T[nb:] = rng.integers(0, K, n_solvent)
    chi = np.zeros((K, K))
    for a in range(K):
        for b in range(K):
            if a != b:
                chi[a, b] = chi_ab * (1.0 + 0.25 * ((a + b) % 3))
    R = _rows3(wrap_f32(pos, Lt))
    V = _rows3(maxwell(rng, N).astype(np.float32))
    return System("small", R, V, T, np.arange(N, dtype=np.int32),
                  chain_bonds(n_chains, chain_len, N), Lt, Mt, K, 1.0, inv_kappa,
                  chi, 100.0, 0.0, 0.03, {"seed": seed})


def permuted(sys: System, seed: int = 99) -> tuple:
    """The same system with beads stored in a random order (bond table remapped)."""
    rng = np.random.default_rng(seed)
    N = sys.N
    perm = rng.permutation(N)          # new position p holds old bead perm[p]
    inv = np.empty(N, dtype=np.int64)
    inv[perm] = np.arange(N)
    b_old = sys.bonds[:, perm]
    b_new = np.where(b_old >= 0, inv[np.maximum(b_old, 0)], -1).astype(np.int32)
    out = System(sys.name + "_perm", sys.R[perm].copy(), sys.V[perm].copy(), sys.T[perm].copy(),
                 sys.tag[perm].copy(), b_new, sys.L, sys.M, sys.K, sys.kT, sys.inv_kappa,
                 sys.chi, sys.k_bond, sys.r0, sys.dt, dict(sys.meta))
    if sys.angles is not None:
        a_old = sys.angles[:, perm]
        idx_rows = (np.arange(a_old.shape[0]) % 3 != 2)[:, None]
        out.angles = np.where(idx_rows, np.where(a_old >= 0, inv[np.maximum(a_old, 0)], -1),
                              a_old).astype(np.int32)
        out.angle_k, out.angle_theta0, out.angle_form = sys.angle_k, sys.angle_theta0, sys.angle_form
    return out, perm


# ---------------------------------------------------------------------------
# A five-species lipid-like system in water, standing in for the paper's own
# MD-SCF workload (coarse-grained phospholipids in water, whose force-field
# parameters are not available here): 12-bead two-tailed lipids
#
#     N - P - G1 - C - C - C - C          species: N = 0 (choline-like head),
#             |                                    P = 1 (phosphate-like),
#             G2 - C - C - C - C                   G = 2 (glycerol), C = 3 (tail),
#                                                  W = 4 (water, single beads)
#
# drawn as branched random walks of bond length 0.97 from uniform random start
# points, plus uniformly placed water, at bead density 3. Bonds are harmonic
# (k = 100, r0 = 0.5, the paper's U = k (r - r0)^2); the glycerol bead G1 has
# three partners, so the bond table has three rows. Angles: P-G1-G2 and
# P-G1-C (type 0, harmonic in theta, theta0 = 120 degrees, k = 12) and the tail
# angles G-C-C and C-C-C (type 1, harmonic in cos theta, theta0 = 180 degrees,
# k = 12). The chi matrix (kT units) makes tails repel water and heads:
# chi_CW = 7, chi_NC = chi_PC = 5, chi_GC = chi_GW = 3, chi_NG = chi_PG = 1.5,
# chi_NP = 0.5, heads and water mutually 0. These values are chosen for the
# benchmark's shape and are not the paper's.
LIPID_BONDS = [(0, 1), (1, 2), (2, 3), (2, 4), (4, 5), (5, 6), (6, 7),
               (3, 8), (8, 9), (9, 10), (10, 11)]
LIPID_TYPES = [0, 1, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3]
LIPID_ANGLES = [((1, 2, 3), 0), ((1, 2, 4), 0), ((2, 4, 5), 1), ((4, 5, 6), 1), ((5, 6, 7), 1),
                ((2, 3, 8), 1), ((3, 8, 9), 1), ((8, 9, 10), 1), ((9, 10, 11), 1)]
LIPID_CHI = {(0, 1): 0.5, (0, 2): 1.5, (1, 2): 1.5, (0, 3): 5.0, (1, 3): 5.0, (2, 3): 3.0,
             (3, 4): 7.0, (2, 4): 3.0}


def table_from_pairs(pairs, N: int) -> np.ndarray:
    """Bond table [D, N] (paper's table form) from undirected pairs."""
    nbr = [[] for _ in range(N)]
    for i, j in pairs:
        nbr[i].append(j)
        nbr[j].append(i)
    D = max((len(v) for v in nbr), default=0)
    tab = np.full((D, N), -1, dtype=np.int32)
    for i, v in enumerate(nbr):
        tab[:len(v), i] = v
    return tab


def angle_table(triplets, N: int) -> np.ndarray:
    """Per-bead angle table [3A, N] from (end, middle, end, type) tuples: each member gets a
    slot (partner, partner, role + 2 type); role 1 = middle (partners are the ends), 0 = end
    (first partner = middle, second = the other end)."""
    slots = [[] for _ in range(N)]
    for i, j, k, t in triplets:
        slots[j].append((i, k, 1 + 2 * t))
        slots[i].append((j, k, 2 * t))
        slots[k].append((j, i, 2 * t))
    A = max((len(v) for v in slots), default=0)
    tab = np.full((3 * A, N), -1, dtype=np.int32)
    tab[2::3] = 0
    for b, v in enumerate(slots):
        for a, (p, q, code) in enumerate(v):
            tab[3 * a, b], tab[3 * a + 1, b], tab[3 * a + 2, b] = p, q, code
    return tab


def lipid_system(n_lipids: int, n_water: int, M: int | None = None, seed: int = BASE_SEED + 5,
                 density: float = 3.0) -> System:
    """The five-species lipid-in-water system above (n_lipids * 12 + n_water beads)."""
    rng = np.random.default_rng(seed)
    per = len(LIPID_TYPES)
    nl = n_lipids * per
    N = nl + n_water
    L = (N / density) ** (1.0 / 3.0)
    M = int(math.ceil(L)) if M is None else M
    pos = np.empty((nl, 3))
    step = rng.standard_normal((n_lipids, per, 3))
    step *= 0.97 / np.linalg.norm(step, axis=2, keepdims=True)
    start = rng.random((n_lipids, 3)) * L
    lip = np.empty((n_lipids, per, 3))
    lip[:, 0] = start
    parent = {1: 0, 2: 1, 3: 2, 4: 2, 5: 4, 6: 5, 7: 6, 8: 3, 9: 8, 10: 9, 11: 10}
    for b in range(1, per):
        lip[:, b] = lip[:, parent[b]] + step[:, b]
    pos[:] = lip.reshape(-1, 3)
    if n_water:
        pos = np.concatenate([pos, rng.random((n_water, 3)) * L])
    T = np.empty(N, dtype=np.uint8)
    T[:nl] = np.tile(np.asarray(LIPID_TYPES, dtype=np.uint8), n_lipids)
    T[nl:] = 4
    pairs = [(m * per + i, m * per + j) for m in range(n_lipids) for i, j in LIPID_BONDS]
    trip = [(m * per + i, m * per + j, m * per + k, t) for m in range(n_lipids)
            for (i, j, k), t in LIPID_ANGLES]
    R = _rows3(wrap_f32(pos, L))
    V = _rows3(maxwell(rng, N).astype(np.float32))
    return System("lipid_k5", R, V, T, np.arange(N, dtype=np.int32), table_from_pairs(pairs, N),
                  (L,) * 3, (M,) * 3, 5, 1.0, 10.0, chi_matrix(5, LIPID_CHI), 100.0, 0.5, 0.03,
                  {"seed": seed, "n_lipids": n_lipids, "n_water": n_water},
                  angles=angle_table(trip, N), angle_k=(12.0, 12.0),
                  angle_theta0=(2.0 * math.pi / 3.0, math.pi), angle_form=(0, 1))
