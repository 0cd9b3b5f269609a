"""Independent brute-force evaluations used to pin the FP64 oracle.

Nothing here calls the oracle or the HIP library. The field force is written
as a pair sum over beads with no mesh arrays: substituting the density
assignment, the potential (eq. 4) and the centred difference into the
interpolated force gives

    F_i = -1/(rho0 dV 2^6S) sum_j A[T_i, T_j] sum_{a,b} W_a(i) W_b(j) D(c_i + a, c_j + b)

with A = kT chi + 1/kappa (the constant -1/kappa of eq. 4 has zero gradient)
and D the periodic centred-difference operator,
D(u, w) = sum_d ([w = u + e_d] - [w = u - e_d]) / (2 h_d) along axis d.
The cell weights are recomputed here in numpy float32 arithmetic.
"""
from __future__ import annotations

import numpy as np

ONE = 1 << 16


def cell_weights(x: float, L: float, M: int):
    """Cell index and 1-D fixed-point weights of one coordinate (float32 arithmetic)."""
    s = np.float32(np.float64(M) / np.float64(np.float32(L)))
    u = np.float32(np.float32(x) * s)
    fl = np.floor(u)
    f = np.float32(u - fl)
    q = int(np.floor(np.float64(f) * ONE))
    return int(fl) % M, (ONE - q, q)


def corner_weights(pos, L, M):
    """[(vertex (x, y, z), W_a)] for the 8 corners of a bead's cell."""
    cw = [cell_weights(pos[d], L[d], M[d]) for d in range(3)]
    out = []
    for az in (0, 1):
        for ay in (0, 1):
            for ax in (0, 1):
                v = ((cw[0][0] + ax) % M[0], (cw[1][0] + ay) % M[1], (cw[2][0] + az) % M[2])
                out.append((v, cw[0][1][ax] * cw[1][1][ay] * cw[2][1][az]))
    return out


def D(u, w, L, M):
    """Periodic centred-difference operator: the gradient vector contribution of V(w) at u."""
    g = np.zeros(3)
    for d in range(3):
        h = float(np.float32(L[d])) / M[d]
        up = list(u)
        up[d] = (u[d] + 1) % M[d]
        dn = list(u)
        dn[d] = (u[d] - 1) % M[d]
        if tuple(up) == tuple(w):
            g[d] += 1.0 / (2 * h)
        if tuple(dn) == tuple(w):
            g[d] -= 1.0 / (2 * h)
    return g


def pair_field_forces(pos, types, L, M, kT, inv_kappa, chi):
    """Field forces of a handful of beads by the pair-sum formula above."""
    N = len(pos)
    vol = np.prod([float(np.float32(x)) for x in L])
    rho0_dV = N / float(np.prod(M))          # rho0 * dV = N / M^3
    A = kT * np.asarray(chi, dtype=np.float64) + inv_kappa
    cw = [corner_weights(p, L, M) for p in pos]
    F = np.zeros((N, 3))
    for i in range(N):
        for j in range(N):
            a_ij = A[types[i], types[j]]
            for (u, wa) in cw[i]:
                for (w, wb) in cw[j]:
                    F[i] -= a_ij * wa * wb * D(u, w, L, M)
    del vol
    return F / (rho0_dV * float(ONE) ** 6)


def dimer_closed_form(d0: float, u0: float, omega2: float, dt: float, n: int):
    """Velocity Verlet on x'' = -omega2 x after n steps, in closed form.

    One step is the linear map [[c, dt], [-omega2 dt (1 + c) / 2, c]] with
    c = 1 - omega2 dt^2 / 2; its determinant is 1 and its trace 2c, so with
    cos(theta) = c its n-th power is cos(n theta) I + sin(n theta)/sin(theta) (M - c I).
    """
    c = 1.0 - omega2 * dt * dt / 2.0
    th = np.arccos(c)
    sn = np.sin(n * th) / np.sin(th)
    x = np.cos(n * th) * d0 + sn * dt * u0
    v = np.cos(n * th) * u0 - sn * omega2 * dt * (1.0 + c) / 2.0 * d0
    return x, v
