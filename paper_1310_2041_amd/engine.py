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
N_ROWS = 6


class HpfState:
    """One periodic system on the GPU: beads, bond table, mesh buffers."""

    def __init__(self, R, Vel, T, tag, bonds, L, M, K, kT, inv_kappa, chi, k_bond, r0, dt,
                 device="cuda", sort_brick=8, halo=1):
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
        self.B = int(sort_brick)
        self.halo = int(halo)
        self.sorted = False      # storage order comes from hpf_sort_by_cell
        nm = self.mesh.M[0] * self.mesh.M[1] * self.mesh.M[2]
        self.nm = nm

        def up(a, dtype):
            return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype).contiguous()

        self.R = up(R, torch.float32)
        self.Vel = up(Vel, torch.float32)
        self.T = up(T, torch.uint8)
        self.tag = up(tag, torch.int32)
        self.bonds = up(bonds, torch.int32) if bonds is not None and len(bonds) else \
            torch.zeros((0, self.N), dtype=torch.int32, device=dev)
        self.F = torch.zeros((self.N, 4), dtype=torch.float32, device=dev)
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
        # the cell-list scatter needs every mesh edge >= B + 1 + 2*halo (0 bytes = unsupported)
        ws = hpf.hpf_scatter_workspace_bytes(self.N, self.mesh, self.K, self.B, self.halo)
        self.cells_ok = ws > 0
        self.scatter_work = torch.empty(max(ws, 1), dtype=torch.uint8, device=dev)
        # mesh buffers; counts start at zero and are cleared by the potential pass
        self.counts = torch.zeros((self.K, nm), dtype=torch.int64, device=dev)
        self.V = torch.empty((self.K, nm), dtype=torch.float32, device=dev)
        self.G = torch.empty((self.K, nm, 4), dtype=torch.float32, device=dev)
        self.part = torch.zeros((N_ROWS, hpf.HPF_NPART), dtype=torch.float64, device=dev)
        self.energy = torch.zeros(8, dtype=torch.float64, device=dev)
        self.steps_done = 0

    @classmethod
    def from_system(cls, s, **kw):
        return cls(s.R, s.V, s.T, s.tag, s.bonds, s.L, s.M, s.K, s.kT, s.inv_kappa, s.chi,
                   s.k_bond, s.r0, s.dt, **kw)

    # ---------------------------------------------------------------- pieces

    def sort(self, stream=None):
        D = self.bonds.shape[0]
        hpf.hpf_sort_by_cell(self.mesh, self.B, self.R, self.Vel, self.T, self.tag,
                             self.bonds if D else None, self.R2, self.Vel2, self.T2, self.tag2,
                             self.bonds2 if D else None, self.work, cell_start=self.cell_start,
                             stream=stream)
        self.R, self.R2 = self.R2, self.R
        self.Vel, self.Vel2 = self.Vel2, self.Vel
        self.T, self.T2 = self.T2, self.T
        self.tag, self.tag2 = self.tag2, self.tag
        self.bonds, self.bonds2 = self.bonds2, self.bonds
        self.sorted = True

    def scatter(self, stream=None):
        """Density counts: cell-list owner tiles when sorted, else the generic scatter."""
        if self.sorted and self.cells_ok:
            hpf.hpf_density_scatter_cells(self.R, self.T, self.mesh, self.K, self.cell_start, self.B,
                                          self.halo, self.counts, self.scatter_work, stream)
        else:
            hpf.hpf_density_scatter(self.R, self.T, self.mesh, self.K, self.counts, stream)

    def field_forces(self, report=False, stream=None):
        """F = field force (scatter, potential, gradient, gather)."""
        self.scatter(stream)
        hpf.hpf_field_potential(self.counts, self.mesh, self.field, self.V,
                                self.part[ROW_W] if report else None, stream)
        hpf.hpf_field_gradient(self.V, self.mesh, self.K, self.G, stream)
        hpf.hpf_force_gather(self.R, self.T, self.mesh, self.K, self.G, self.F, stream)

    def bond_forces(self, report=False, stream=None):
        hpf.bond_forces(self.R, self.bonds if self.bonds.shape[0] else None, self.k_bond, self.r0,
                        self.box, self.F, self.part[ROW_EB] if report else None, stream)

    def forces(self, report=False, stream=None):
        self.field_forces(report, stream)
        self.bond_forces(report, stream)

    def step(self, report=False, sort=False, stream=None):
        hpf.verlet_step(self.R, self.Vel, self.F, self.dt, self.box, 1, stream=stream)
        if sort:
            self.sort(stream)
        self.forces(report, stream)
        hpf.verlet_step(None, self.Vel, self.F, self.dt, self.box, 2,
                        kin_part=self.part[ROW_KE:ROW_KE + 4] if report else None, stream=stream)
        if report:
            hpf.hpf_reduce_partials(self.part, N_ROWS, self.energy, stream)
        self.steps_done += 1

    def start(self, sort=True, stream=None):
        """Initial sort and force evaluation, with energies of the initial state."""
        if sort:
            self.sort(stream)
        self.forces(report=True, stream=stream)
        hpf.verlet_step(None, self.Vel, torch.zeros_like(self.F), self.dt, self.box, 2,
                        kin_part=self.part[ROW_KE:ROW_KE + 4], stream=stream)
        hpf.hpf_reduce_partials(self.part, N_ROWS, self.energy, stream)

    # ------------------------------------------------------------ fused path

    def prime(self, stream=None):
        """First half step after start(): (x_0, v_0, F_0) -> (x_1, v_1/2)."""
        hpf.verlet_step(self.R, self.Vel, self.F, self.dt, self.box, 1, stream=stream)

    def step_fused(self, report=False, sort=False, stream=None):
        """(x_n, v_n-1/2) -> (x_n+1, v_n+1/2) with hpf_advance; energies of step n.

        Bitwise equal to step() followed by the next step's first half step."""
        if sort:
            self.sort(stream)
        self.scatter(stream)
        hpf.hpf_field_potential(self.counts, self.mesh, self.field, self.V,
                                self.part[ROW_W] if report else None, stream)
        hpf.hpf_field_gradient(self.V, self.mesh, self.K, self.G, stream)
        hpf.hpf_advance(self.R, self.R2, self.Vel, self.T, self.mesh, self.K, self.G,
                        self.bonds if self.bonds.shape[0] else None, self.k_bond, self.r0, self.box,
                        self.dt, e_part=self.part[ROW_EB] if report else None,
                        kin_part=self.part[ROW_KE:ROW_KE + 4] if report else None, stream=stream)
        self.R, self.R2 = self.R2, self.R
        if report:
            hpf.hpf_reduce_partials(self.part, N_ROWS, self.energy, stream)
        self.steps_done += 1

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
        return {"KE": ke, "E_bond": eb, "W": w, "E_tot": ke + eb + w, "P": e[3:6].copy()}

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
