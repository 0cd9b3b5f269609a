"""Device-resident state of one hPF-MD system and the timestep built from the
C-ABI calls (velocity Verlet around a density-field force evaluation).

Per step, on one HIP stream:
  verlet_step(half=1)          kick + drift + wrap
  hpf_sort_by_cell             every ``sort_every`` steps (ping-pong buffers)
  hpf_density_scatter          fixed-point CIC counts
  hpf_field_potential          FP64 phi and V, counts cleared
  hpf_field_gradient           centred mesh gradient
  hpf_force_gather             F = field force (overwrite)
  bond_forces                  F += harmonic bonds
  verlet_step(half=2)          kick, FP64 kinetic-energy partials
Energies are reduced in FP64 only on reporting steps.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hpf

# rows of the partial-sum buffer
ROW_W, ROW_EB, ROW_KE = 0, 1, 2      # KE, Px, Py, Pz occupy rows 2..5
ROW_EA = 6                           # angle energy
N_ROWS = 7


LDS_BYTES = 160 * 1024
RESORT_MIN_BRICKS = 8192


def auto_brick(M, K: int, halo: int) -> int:
    """Sort brick edge for the fused depositing pass: 16 cells when the mesh holds at least
    512 such bricks (two per CU) and their deposit box of K (17 + 2 halo)^3 uint64 fits in
    LDS, else 8. Larger bricks halve the partial-box traffic (the box overhang is a smaller
    share of the brick); on small meshes they would leave CUs idle."""
    B = 16
    P = B + 1 + 2 * halo
    nb = 1
    for d in range(3):
        nb *= -(-int(M[d]) // B)
    if nb >= 512 and K * P ** 3 * 8 <= LDS_BYTES and all(int(m) >= P for m in M):
        return B
    return 8


class HpfState:
    """One periodic system on the GPU: beads, bond table, mesh buffers."""

    def __init__(self, R, Vel, T, tag, bonds, L, M, K, kT, inv_kappa, chi, k_bond, r0, dt,
                 device="cuda", sort_brick=0, halo=1, advance="scatter",
                 field_every=1, stencil="centred", angles=None, angle_k=(), angle_theta0=(),
                 angle_form=(), composition_list=False):
        dev = torch.device(device)
        self.N = int(R.shape[0])
        self.K = int(K)
        self.dt = float(dt)
        self.k_bond = float(k_bond)
        self.r0 = float(r0)
        self.L = tuple(float(x) for x in (L if hasattr(L, "__len__") else (L,) * 3))
        self.mesh = hpf.hpf_mesh_make(self.L, M, self.N)
        self.field = hpf.make_field(self.K, kT, inv_kappa, chi)
        self.box = self.L
        # 0 = auto_brick(): 16-cell bricks on large meshes, else 8
        self.B = int(sort_brick) or auto_brick(self.mesh.M, self.K, int(halo))
        self.halo = int(halo)
        # How the fused step advances cell-sorted beads: "scatter" = hpf_advance_scatter (also
        # deposits x_n+1, so the next step only finishes the density), "plain" = hpf_advance.
        # Unsorted beads always take hpf_advance.
        self.advance_mode = advance
        # Force interpolation (Algorithm 1 Kernels 3-4): "centred" = centred differences at the
        # mesh points gathered with the deposit's weights (hpf_field_gradient +
        # hpf_force_gather, and the fused passes); "staggered" = the paper-literal backward /
        # forward differences at the nearest mesh point (hpf_force_gather_staggered; the
        # six-call step only).
        if stencil not in ("centred", "staggered"):
            raise ValueError("stencil must be 'centred' or 'staggered'")
        self.stencil = stencil
        # Field-update interval (MD-SCF section): the density field (counts, V, G) is rebuilt
        # at force evaluations whose index is a multiple of field_every (evaluation 0 is
        # start(), evaluation s comes after step s); the others gather from the last G, and
        # the reported W is the last rebuild's.
        if int(field_every) < 1:
            raise ValueError("field_every must be >= 1")
        self.field_every = int(field_every)
        # The composition list leaves the gradient of an absent species stale at a mesh point.
        # That is exact only when every bead gathers at the positions that built the counts
        # (each corner it reaches with a non-zero weight then holds its own species), i.e. the
        # field is rebuilt at every force evaluation and gathered with the deposit's weights.
        if composition_list and (self.field_every != 1 or stencil != "centred"):
            raise ValueError("composition_list needs field_every=1 and the centred stencil")
        self.density_pending = False   # partial boxes + counts hold the deposit of the current R
        # when True, the fused passes also store the total force at x_n into F (F_out)
        self.keep_force = False
        # Andersen thermostat (set_thermostat): (p, kT, seed) and the device time level
        self.thermo = None
        self.tstep = None
        self.sorted = False      # storage order comes from hpf_sort_by_cell
        nm = self.mesh.M[0] * self.mesh.M[1] * self.mesh.M[2]
        self.nm = nm

        def up(a, dtype):
            return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype).contiguous()

        # bead rows are (x, y, z), 12 bytes; (N, 4) host arrays give their first three columns
        self.R = up(np.asarray(R)[:, :3], torch.float32)
        self.Vel = up(np.asarray(Vel)[:, :3], torch.float32)
        self.T = up(T, torch.uint8)
        self.tag = up(tag, torch.int32)
        self.bonds = up(bonds, torch.int32) if bonds is not None and len(bonds) else \
            torch.zeros((0, self.N), dtype=torch.int32, device=dev)
        self.F = torch.zeros((self.N, 3), dtype=torch.float32, device=dev)
        # angles (Bonded forces section): per-bead table [3A, N] and per-type parameters; the
        # six-call step evaluates them (the fused passes take bonds only)
        self.angles = up(angles, torch.int32) if angles is not None and len(angles) else None
        self.angles2 = torch.empty_like(self.angles) if self.angles is not None else None
        self.angle_params = (tuple(angle_k), tuple(angle_theta0), tuple(angle_form))
        # ping-pong targets of the cell sort
        self.R2 = torch.empty_like(self.R)
        self.Vel2 = torch.empty_like(self.Vel)
        self.T2 = torch.empty_like(self.T)
        self.tag2 = torch.empty_like(self.tag)
        self.bonds2 = torch.empty_like(self.bonds)
        self.work = torch.empty(hpf.hpf_sort_workspace_bytes(self.N, self.mesh, self.B),
                                dtype=torch.uint8, device=dev)
        self.cell_start = torch.empty(hpf.sort_key_count(self.mesh, self.B) + 2,
                                      dtype=torch.int32, device=dev)
        self.cell_start2 = torch.empty_like(self.cell_start)
        # Re-sort from the previous sort's order (hpf_resort_by_cell) once sorted. Its passes
        # run one workgroup per brick, so it pays on meshes of many bricks (10^8 beads in
        # 32,768 bricks: 7 ms against 40 ms for the full sort); with a few hundred large
        # bricks the full sort is faster (0.48 against 0.84 ms for 10^7 beads in 512).
        self.resort = hpf.sort_key_count(self.mesh, self.B) >= RESORT_MIN_BRICKS
        # the cell-list scatter needs every mesh edge >= B + 1 + 2*halo (0 bytes = unsupported)
        ws = hpf.hpf_scatter_workspace_bytes(self.N, self.mesh, self.K, self.B, self.halo)
        self.cells_ok = ws > 0
        self.scatter_work = torch.empty(max(ws, 1), dtype=torch.uint8, device=dev)
        # mesh buffers; counts start at zero and are cleared by the potential pass
        self.counts = torch.zeros((self.K, nm), dtype=torch.int64, device=dev)
        self.V = torch.empty((self.K, nm), dtype=torch.float32, device=dev)
        # Composition list (MD-SCF section): the potential pass records which species are
        # present at each mesh point and the gradient pass skips the absent ones; G starts at
        # zero so that entries never written stay finite.
        self.present = torch.zeros(nm, dtype=torch.uint8, device=dev) if composition_list else None
        self.G = (torch.zeros if composition_list else torch.empty)((self.K, nm, 3), dtype=torch.float32,
                                                                    device=dev)
        self.part = torch.zeros((N_ROWS, hpf.HPF_NPART), dtype=torch.float64, device=dev)
        self.energy = torch.zeros(8, dtype=torch.float64, device=dev)
        self.steps_done = 0

    def set_thermostat(self, rate: float, kT: float | None = None, seed: int = 1, tag_offset: int = 0):
        """NVT with the Andersen thermostat (Integration methods section): every step each bead
        collides with probability rate * dt and takes a Maxwell velocity at kT (the field's kT
        by default). The time level of the collisions lives on the device and advances with
        every step, so graph replays draw fresh numbers. rate = 0 returns to NVE. tag_offset is
        added to the tags in the generator's counter (a replica of a batch numbers its tags from
        its first bead on)."""
        p = float(rate) * self.dt
        if p == 0.0:
            self.thermo = None
            return
        if not 0.0 < p <= 1.0:
            raise ValueError("rate * dt must lie in (0, 1]")
        self.thermo = (p, float(self.field.kT if kT is None else kT), int(seed), int(tag_offset))
        self.tstep = torch.tensor([self.steps_done + 1], dtype=torch.int64, device=self.R.device)

    def thermostat(self):
        """The C thermostat description for the current storage order (None for NVE)."""
        if self.thermo is None:
            return None
        p, kT, seed, tag_offset = self.thermo
        return hpf.make_thermostat(p, kT, seed, self.tstep, self.tag, tag_offset)

    _SWAPPED = ("R", "R2", "Vel", "Vel2", "T", "T2", "tag", "tag2", "bonds", "bonds2", "cell_start",
                "cell_start2", "angles", "angles2")

    def snapshot(self) -> dict:
        """The host-side stepping state (which buffers are current, the step count, whether a
        deposit is pending), so that a caller that replays captured steps can put the object
        back in step with the device."""
        d = {k: getattr(self, k) for k in self._SWAPPED}
        d.update(steps_done=self.steps_done, density_pending=self.density_pending,
                 sorted=self.sorted)
        return d

    def restore(self, d: dict):
        for k, v in d.items():
            setattr(self, k, v)

    @classmethod
    def from_system(cls, s, **kw):
        if getattr(s, "angles", None) is not None:
            kw = dict(dict(angles=s.angles, angle_k=s.angle_k, angle_theta0=s.angle_theta0,
                           angle_form=s.angle_form), **kw)
        return cls(s.R, s.V, s.T, s.tag, s.bonds, s.L, s.M, s.K, s.kT, s.inv_kappa, s.chi,
                   s.k_bond, s.r0, s.dt, **kw)

    # ---------------------------------------------------------------- pieces

    def sort(self, stream=None):
        """Canonical (brick, tag) order. From the order of an earlier sort the incremental
        re-sort builds the same order brick by brick; otherwise the full counting sort."""
        D = self.bonds.shape[0]
        if self.sorted and self.resort:
            hpf.hpf_resort_by_cell(self.mesh, self.B, self.R, self.Vel, self.T, self.tag,
                                   self.bonds if D else None, self.R2, self.Vel2, self.T2, self.tag2,
                                   self.bonds2 if D else None, self.work, self.cell_start, self.cell_start2,
                                   stream=stream)
            self.cell_start, self.cell_start2 = self.cell_start2, self.cell_start
        else:
            hpf.hpf_sort_by_cell(self.mesh, self.B, self.R, self.Vel, self.T, self.tag,
                                 self.bonds if D else None, self.R2, self.Vel2, self.T2, self.tag2,
                                 self.bonds2 if D else None, self.work, cell_start=self.cell_start,
                                 stream=stream)
        self.R, self.R2 = self.R2, self.R
        self.Vel, self.Vel2 = self.Vel2, self.Vel
        self.T, self.T2 = self.T2, self.T
        self.tag, self.tag2 = self.tag2, self.tag
        self.bonds, self.bonds2 = self.bonds2, self.bonds
        if self.angles is not None:
            hpf.hpf_sort_angles(self.mesh, self.B, self.angles, self.angles2, self.work, stream)
            self.angles, self.angles2 = self.angles2, self.angles
        self.sorted = True

    def scatter(self, stream=None):
        """Density counts: cell-list owner tiles when sorted, else the generic scatter."""
        self.density_pending = False
        if self.sorted and self.cells_ok:
            hpf.hpf_density_scatter_cells(self.R, self.T, self.mesh, self.K, self.cell_start, self.B,
                                          self.halo, self.counts, self.scatter_work, stream)
        else:
            hpf.hpf_density_scatter(self.R, self.T, self.mesh, self.K, self.counts, stream)

    def rebuilds_field(self, evaluation: int) -> bool:
        """Whether force evaluation `evaluation` rebuilds the density field."""
        return evaluation % self.field_every == 0

    def field_forces(self, report=False, stream=None, rebuild=True):
        """F = field force (scatter, potential, gradient, gather); without `rebuild`, only the
        gather from the last gradient. W partials are kept whenever the interval exceeds one,
        so that the steps until the next rebuild report the field energy in force."""
        if rebuild:
            self.scatter(stream)
            hpf.hpf_field_potential(self.counts, self.mesh, self.field, self.V,
                                    self.part[ROW_W] if (report or self.field_every > 1) else None,
                                    stream, present=self.present)
            if self.stencil == "centred":
                hpf.hpf_field_gradient(self.V, self.mesh, self.K, self.G, stream, present=self.present)
        if self.stencil == "staggered":
            hpf.hpf_force_gather_staggered(self.R, self.T, self.mesh, self.K, self.V, self.F, stream)
        else:
            hpf.hpf_force_gather(self.R, self.T, self.mesh, self.K, self.G, self.F, stream)

    def bond_forces(self, report=False, stream=None):
        hpf.bond_forces(self.R, self.bonds if self.bonds.shape[0] else None, self.k_bond, self.r0,
                        self.box, self.F, self.part[ROW_EB] if report else None, stream)

    def angle_forces(self, report=False, stream=None):
        if self.angles is None:
            return
        k, th, fm = self.angle_params
        hpf.angle_forces(self.R, self.angles, k, th, fm, self.box, self.F,
                         self.part[ROW_EA] if report else None, stream)

    def forces(self, report=False, stream=None, rebuild=True):
        self.field_forces(report, stream, rebuild)
        self.bond_forces(report, stream)
        self.angle_forces(report, stream)

    def step(self, report=False, sort=False, stream=None):
        self.density_pending = False
        hpf.verlet_step(self.R, self.Vel, self.F, self.dt, self.box, 1, stream=stream)
        if sort:
            self.sort(stream)
        self.forces(report, stream, rebuild=self.rebuilds_field(self.steps_done + 1))
        kin = self.part[ROW_KE:ROW_KE + 4] if report else None
        th = self.thermostat()
        hpf.verlet_step(None, self.Vel, self.F, self.dt, self.box, 2,
                        kin_part=kin if th is None else None, stream=stream)
        if th is not None:
            hpf.hpf_andersen(self.Vel, th, kin_part=kin, stream=stream)
            self._advance_time_level(stream)
        if report:
            hpf.hpf_reduce_partials(self.part, N_ROWS, self.energy, stream)
        self.steps_done += 1

    def _advance_time_level(self, stream=None):
        if stream is None:
            self.tstep.add_(1)
        else:
            with torch.cuda.stream(stream if isinstance(stream, torch.cuda.Stream) else
                                   torch.cuda.ExternalStream(int(stream))):
                self.tstep.add_(1)

    def start(self, sort=True, stream=None):
        """Initial sort and force evaluation, with energies of the initial state."""
        self.density_pending = False
        if sort:
            self.sort(stream)
        self.forces(report=True, stream=stream)
        hpf.verlet_step(None, self.Vel, torch.zeros_like(self.F), self.dt, self.box, 2,
                        kin_part=self.part[ROW_KE:ROW_KE + 4], stream=stream)
        hpf.hpf_reduce_partials(self.part, N_ROWS, self.energy, stream)

    # ------------------------------------------------------------ fused path

    def prime(self, stream=None):
        """First half step after start(): (x_0, v_0, F_0) -> (x_1, v_1/2)."""
        self.density_pending = False
        hpf.verlet_step(self.R, self.Vel, self.F, self.dt, self.box, 1, stream=stream)

    def step_fused(self, report=False, sort=False, stream=None):
        """(x_n, v_n-1/2) -> (x_n+1, v_n+1/2) with hpf_advance; energies of step n.
        The fused passes interpolate with the centred stencil only.

        Bitwise equal to step() followed by the next step's first half step."""
        if self.stencil != "centred" or self.angles is not None:
            raise ValueError("the fused passes take the centred stencil and bonds only; "
                             "step() runs the staggered stencil and angles")
        if sort:
            self.sort(stream)
        # this step's force evaluation is number steps_done + 1 (start() was number 0)
        if self.rebuilds_field(self.steps_done + 1):
            self.potential(report or self.field_every > 1, stream)
            hpf.hpf_field_gradient(self.V, self.mesh, self.K, self.G, stream, present=self.present)
        self.advance(report, stream, deposit=self.rebuilds_field(self.steps_done + 2))
        if report:
            hpf.hpf_reduce_partials(self.part, N_ROWS, self.energy, stream)
        self.steps_done += 1

    def potential(self, report=False, stream=None):
        """Counts and potential of the current positions: finish the deposit the last fused
        pass made and form V in one pass, or scatter from scratch and then form V."""
        w = self.part[ROW_W] if report else None
        if self.density_pending:
            hpf.hpf_field_potential_cells(self.counts, self.N, self.mesh, self.field, self.B, self.halo,
                                          self.scatter_work, self.V, w, stream, present=self.present)
            self.density_pending = False
        else:
            self.scatter(stream)
            hpf.hpf_field_potential(self.counts, self.mesh, self.field, self.V, w, stream, present=self.present)

    def uses_scatter_advance(self) -> bool:
        return self.advance_mode == "scatter" and self.sorted and self.cells_ok

    def advance(self, report=False, stream=None, deposit=True):
        """Fused forces + Verlet pass, x_n -> x_n+1 (with the density deposit of x_n+1 when
        cell-sorted). Counts must be zero on entry (the potential pass
        leaves them so). Without `deposit` (the next step keeps the field) the plain pass runs
        instead of the depositing one; the beads move the same either way."""
        bonds = self.bonds if self.bonds.shape[0] else None
        e_part = self.part[ROW_EB] if report else None
        kin_part = self.part[ROW_KE:ROW_KE + 4] if report else None
        F_out = self.F if self.keep_force else None
        th = self.thermostat()
        self.density_pending = False
        if deposit and self.uses_scatter_advance():
            hpf.hpf_advance_scatter(self.R, self.R2, self.Vel, self.T, self.mesh, self.K, self.G, bonds,
                                    self.k_bond, self.r0, self.box, self.dt, self.cell_start, self.B,
                                    self.halo, self.counts, self.scatter_work, F_out=F_out, e_part=e_part,
                                    kin_part=kin_part, thermostat=th, stream=stream)
            self.density_pending = True
        else:
            hpf.hpf_advance(self.R, self.R2, self.Vel, self.T, self.mesh, self.K, self.G, bonds,
                            self.k_bond, self.r0, self.box, self.dt, F_out=F_out, e_part=e_part,
                            kin_part=kin_part, thermostat=th, stream=stream)
        if th is not None:
            self._advance_time_level(stream)
        self.R, self.R2 = self.R2, self.R

    def run_fused(self, n_steps, report_every=0, sort_every=10, stream=None):
        out = []
        for i in range(n_steps):
            rep = report_every > 0 and (i + 1) % report_every == 0
            self.step_fused(report=rep, sort=sort_every > 0 and (self.steps_done % sort_every == 0),
                            stream=stream)
            if rep:
                out.append(self.energies())
        return out

    def energies(self) -> dict:
        """{KE, E_bond, W, E_tot, P} of the last reporting step (synchronises)."""
        e = self.energy.cpu().numpy()
        ke, eb, w = e[ROW_KE], e[ROW_EB], e[ROW_W]
        ea = e[ROW_EA] if self.angles is not None else 0.0
        return {"KE": ke, "E_bond": eb, "W": w, "E_angle": ea, "E_tot": ke + eb + w + ea,
                "P": e[3:6].copy()}

    def run(self, n_steps, report_every=0, sort_every=10, stream=None):
        out = []
        for i in range(n_steps):
            rep = report_every > 0 and (i + 1) % report_every == 0
            self.step(report=rep, sort=sort_every > 0 and (self.steps_done % sort_every == 0),
                      stream=stream)
            if rep:
                out.append(self.energies())
        return out

    def host_beads(self):
        """(R, Vel, T, tag, bonds) as numpy arrays, in current storage order."""
        return (self.R.cpu().numpy(), self.Vel.cpu().numpy(), self.T.cpu().numpy(),
                self.tag.cpu().numpy(), self.bonds.cpu().numpy())


# ------------------------------------------------------------------ batches

class BatchState:
    """Many replicas advanced together through the batched entry points.

    Replicas are concatenated in the given order: beads (global bond indices
    and tags), and meshes. Each replica keeps its own box, mesh and chi; K,
    bond parameters and dt are shared.
    """

    def __init__(self, systems, sort_every=10, brick=8, halo=1, bead_chunk=4096,
                 mesh_chunk=16384, fuse_deposit=True, device="cuda", thermostat_rate=0.0,
                 thermostat_seed=1):
        dev = torch.device(device)
        s0 = systems[0]
        self.K = int(s0.K)
        self.D = int(s0.bonds.shape[0])
        self.n_rep = len(systems)
        offs = np.cumsum([0] + [s.N for s in systems])
        self.offsets = offs
        self.Ntot = int(offs[-1])
        R = np.concatenate([s.R for s in systems])
        V = np.concatenate([s.V for s in systems])
        T = np.concatenate([s.T for s in systems])
        tag = np.arange(self.Ntot, dtype=np.int32)
        bonds = np.concatenate([np.where(s.bonds >= 0, s.bonds + o, -1).astype(np.int32)
                                for s, o in zip(systems, offs[:-1])], axis=1)

        def up(a, dtype):
            return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype).contiguous()

        self.R = [up(R[:, :3], torch.float32), torch.empty((self.Ntot, 3), dtype=torch.float32, device=dev)]
        self.Vel = [up(V[:, :3], torch.float32), torch.empty((self.Ntot, 3), dtype=torch.float32, device=dev)]
        self.T = [up(T, torch.uint8), torch.empty(self.Ntot, dtype=torch.uint8, device=dev)]
        self.tag = [up(tag, torch.int32), torch.empty(self.Ntot, dtype=torch.int32, device=dev)]
        self.bonds = [up(bonds, torch.int32), torch.empty_like(up(bonds, torch.int32))]
        self.nm = [int(np.prod(s.M)) for s in systems]
        nm_tot = sum(self.nm)
        self.counts = torch.zeros(self.K * nm_tot, dtype=torch.int64, device=dev)
        self.V = torch.empty(self.K * nm_tot, dtype=torch.float32, device=dev)
        self.G = torch.empty(self.K * nm_tot * 3, dtype=torch.float32, device=dev)
        reps = []
        for s, o in zip(systems, offs[:-1]):
            r = hpf.Replica()
            r.bead_offset = int(o)
            r.n_beads = s.N
            r.L[:] = [float(x) for x in s.L]
            r.M[:] = [int(x) for x in s.M]
            r.kT = float(s.kT)
            r.inv_kappa = float(s.inv_kappa)
            for a in range(self.K):
                for b in range(self.K):
                    r.chi[a * self.K + b] = float(s.chi[a][b])
            reps.append(r)
        self.reps = reps
        cfg = hpf.BatchConfig()
        cfg.K, cfg.D = self.K, self.D
        cfg.k_bond, cfg.r0, cfg.dt = float(s0.k_bond), float(s0.r0), float(s0.dt)
        cfg.brick, cfg.halo, cfg.sort_every = brick, halo, sort_every
        cfg.bead_chunk, cfg.mesh_chunk = bead_chunk, mesh_chunk
        cfg.fuse_deposit = int(fuse_deposit)
        # Andersen thermostat: collision probability per step, each replica at its own kT
        cfg.thermo_p = float(thermostat_rate) * float(s0.dt)
        cfg.thermo_seed = int(thermostat_seed)
        self.cfg = cfg
        ws = hpf.hpf_batch_workspace_bytes(reps, cfg)
        if ws == 0:
            raise ValueError("batch sizes not supported (mesh edges must be >= brick + 5)")
        self.work = torch.empty(ws, dtype=torch.uint8, device=dev)
        bufs = hpf.BatchBuffers()
        for i in range(2):
            bufs.R[i] = self.R[i].data_ptr()
            bufs.Vel[i] = self.Vel[i].data_ptr()
            bufs.T[i] = self.T[i].data_ptr()
            bufs.tag[i] = self.tag[i].data_ptr()
            bufs.bonds[i] = self.bonds[i].data_ptr() if self.D else None
        bufs.counts = self.counts.data_ptr()
        bufs.V = self.V.data_ptr()
        bufs.G = self.G.data_ptr()
        self.bufs = bufs
        self.handle = hpf.hpf_batch_create(reps, cfg, bufs, self.work)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            hpf.hpf_batch_destroy(h)
            self.handle = None

    def start(self, stream=None):
        hpf.hpf_batch_start(self.handle, stream)

    def step(self, n=1, report_last=True, stream=None):
        hpf.hpf_batch_step(self.handle, n, report_last, stream)

    def density(self, stream=None):
        """Density counts of every replica at the current positions, as a new int64 tensor
        holding uint64 bits (replica r's [K][M_r^3] block follows replica r-1's)."""
        out = torch.empty_like(self.counts)
        hpf.hpf_batch_density(self.handle, out, stream)
        return out

    def tune(self, trial_steps=3, stream=None):
        cfg, ms = hpf.hpf_batch_tune(self.handle, trial_steps, stream)
        self.cfg = cfg
        return {"halo": cfg.halo, "sort_every": cfg.sort_every, "bead_chunk": cfg.bead_chunk,
                "mesh_chunk": cfg.mesh_chunk, "fuse_deposit": cfg.fuse_deposit}, ms

    def _current(self, name):
        ptr = hpf.hpf_batch_current(self.handle)[name]
        for t in getattr(self, name):
            if t.data_ptr() == ptr:
                return t
        raise RuntimeError("unknown current buffer")

    def energies(self) -> np.ndarray:
        """[n_rep, 8] = KE, E_bond, W, E_tot, Px, Py, Pz, 0 of the last reporting step."""
        ptr = hpf.hpf_batch_current(self.handle)["energies"]
        off = ptr - self.work.data_ptr()
        e = self.work[off:off + 64 * self.n_rep].view(torch.float64).reshape(self.n_rep, 8)
        return e.cpu().numpy()

    def replica_beads(self, r):
        """(R, Vel, T, tag - offset, bonds - offset) of replica r, in storage order."""
        a, b = int(self.offsets[r]), int(self.offsets[r + 1])
        R = self._current("R")[a:b].cpu().numpy()
        V = self._current("Vel")[a:b].cpu().numpy()
        T = self._current("T")[a:b].cpu().numpy()
        tag = self._current("tag")[a:b].cpu().numpy() - a
        bonds = self._current("bonds")[:, a:b].cpu().numpy()
        bonds = np.where(bonds >= 0, bonds - a, -1)
        return R, V, T, tag, bonds


class Graph:
    """A HIP graph of whatever library calls `fn` enqueues on a private stream."""

    def __init__(self, fn):
        self.stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(self.stream):
            hpf.hpf_graph_begin(self.stream)
            try:
                fn()
            finally:
                self.handle = hpf.hpf_graph_end(self.stream)

    def launch(self, stream=None):
        """Replay on this graph's own stream, or on `stream`. Replays of several graphs that
        must run one after the other go to one stream: graphs replayed on different streams
        are not ordered with respect to each other."""
        hpf.hpf_graph_launch(self.handle, self.stream if stream is None else stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            torch.cuda.synchronize()
            hpf.hpf_graph_destroy(h)
            self.handle = None
