"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-derived
values, closed forms, invariants, or the independent pair-sum evaluation in
``bruteforce.py``. They run on the CPU only.
"""
import os

import numpy as np
import pytest

import bruteforce as bf
from synth import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TWO48 = 2 ** 48


def _pos4(xyz):
    xyz = np.asarray(xyz, dtype=np.float32).reshape(-1, 3)
    out = np.zeros((xyz.shape[0], 4), dtype=np.float32)
    out[:, :3] = xyz
    return out


def _read_golden_cic():
    cases, cur = [], None
    with open(os.path.join(GOLDEN, "cic_single_bead.txt")) as fh:
        for line in fh:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "case":
                cur = {"L": float(t[2]), "M": int(t[3]), "x": [float(v) for v in t[4:7]],
                       "v": {}}
                cases.append(cur)
            elif t[0] == "v":
                cur["v"][(int(t[1]), int(t[2]), int(t[3]))] = int(t[4])
    return cases


# ---------------------------------------------------------------- O1-O3 ----

def test_golden_single_bead_deposit(oracle_mod):
    """Hand-derived CIC deposits (tests/golden/cic_single_bead.txt)."""
    for case in _read_golden_cic():
        counts, skipped = oracle_mod.density(_pos4(case["x"]), np.zeros(1, np.uint8),
                                             case["L"], case["M"], 1)
        assert skipped == 0
        expect = np.zeros_like(counts)
        for (x, y, z), c in case["v"].items():
            expect[0, z, y, x] = c
        assert np.array_equal(counts, expect)


def test_partition_of_unity_exact(oracle_mod):
    s = wl.small_system(300, 7, (9.3, 7.7, 11.1), (9, 8, 13), K=3, n_solvent=57, seed=3)
    counts, skipped = oracle_mod.density(s.R, s.T, s.L, s.M, s.K)
    assert skipped == 0
    for k in range(s.K):
        assert int(counts[k].sum(dtype=np.uint64)) == int((s.T == k).sum()) * TWO48


def test_cell_weights_match_independent_float32(oracle_mod):
    rng = np.random.default_rng(11)
    for L, M in [(18.8, 20), (69.3, 64), (149.4, 128), (322.0, 256), (4.7, 5)]:
        s = np.float32(np.float64(M) / np.float64(np.float32(L)))
        xs = np.concatenate([rng.random(200) * L, [0.0, np.nextafter(np.float32(L), 0),
                                                   -1e-7, -0.3, L * 1.5]]).astype(np.float32)
        for x in xs:
            bad, c, w = oracle_mod.cell_weights(float(x), s, M)
            assert bad == 0
            c2, w2 = bf.cell_weights(float(x), L, M)
            assert (c, int(w[0]), int(w[1])) == (c2, w2[0], w2[1])


def test_invalid_beads_skipped(oracle_mod):
    R = _pos4([[1.0, 1.0, 1.0], [np.nan, 1.0, 1.0], [1.0, np.inf, 1.0], [1e30, 1.0, 1.0],
               [2.0, 2.0, 2.0]])
    T = np.array([0, 0, 0, 0, 5], dtype=np.uint8)     # type 5 >= K is invalid too
    counts, skipped = oracle_mod.density(R, T, 8.0, 8, 2)
    assert skipped == 4
    assert int(counts.sum(dtype=np.uint64)) == TWO48


def test_permutation_invariance(oracle_mod):
    s = wl.small_system(200, 10, 12.0, 12, seed=5)
    sp, perm = wl.permuted(s)
    c1, _ = oracle_mod.density(s.R, s.T, s.L, s.M, s.K)
    c2, _ = oracle_mod.density(sp.R, sp.T, sp.L, sp.M, sp.K)
    assert np.array_equal(c1, c2)
    F1, Fb1, _ = oracle_mod.forces(s)
    F2, Fb2, _ = oracle_mod.forces(sp)
    assert np.array_equal(F1[perm], F2)
    assert np.array_equal(Fb1[perm], Fb2)


def test_whole_cell_translation(oracle_mod):
    """L = M = 16 (h = 1): shifting every bead by whole cells rolls the counts."""
    rng = np.random.default_rng(2)
    N = 3000
    xyz = np.floor(rng.random((N, 3)) * 16 * 2 ** 16) / 2 ** 16     # exact dyadics
    T = rng.integers(0, 2, N).astype(np.uint8)
    c0, _ = oracle_mod.density(_pos4(xyz), T, 16.0, 16, 2)
    shift = np.array([3, 0, 5])
    xyz2 = np.mod(xyz + shift, 16.0)
    c1, _ = oracle_mod.density(_pos4(xyz2), T, 16.0, 16, 2)
    assert np.array_equal(np.roll(c0, shift=(5, 0, 3), axis=(1, 2, 3)), c1)


# ---------------------------------------------------------------- O4-O5 ----

def test_uniform_melt_potential_and_zero_force(oracle_mod):
    """One A and one B bead at every cell centre: phi_A = phi_B = 1/2, no force."""
    M, L = 16, 16.0
    g = (np.arange(M) + 0.5)
    xyz = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    xyz = np.concatenate([xyz, xyz])
    T = np.repeat(np.array([0, 1], np.uint8), M ** 3)
    chi = np.array([[0.3, 1.2], [1.2, 0.1]])
    kT, ik = 1.3, 7.0
    counts, _ = oracle_mod.density(_pos4(xyz), T, L, M, 2)
    assert np.all(counts == TWO48)
    V, W = oracle_mod.potential(counts, L, M, len(T), kT, ik, chi)
    # eq. 5 with phi_A = phi_B = 1/2 and sum phi = 1
    assert np.allclose(V[0], kT * (0.3 * 0.5 + 1.2 * 0.5), rtol=0, atol=1e-15)
    assert np.allclose(V[1], kT * (1.2 * 0.5 + 0.1 * 0.5), rtol=0, atol=1e-15)
    G = oracle_mod.gradient(V, L, M)
    assert np.all(G == 0.0)
    F = oracle_mod.gather(_pos4(xyz), T, L, M, G)
    assert np.all(F == 0.0)
    # W = rho0 dV * M^3 * [kT/2 * phi.chi.phi + 0]
    phi = np.array([0.5, 0.5])
    assert W == pytest.approx(2.0 * M ** 3 * 0.5 * kT * phi @ chi @ phi, rel=1e-12)  # sum of 4096 terms


def test_two_species_formula_eq5(oracle_mod):
    s = wl.small_system(80, 10, 7.3, 7, seed=8)
    counts, _ = oracle_mod.density(s.R, s.T, s.L, s.M, 2)
    chi = np.array([[0.4, 1.7], [1.7, -0.2]])
    kT, ik = 0.9, 4.5
    V, _ = oracle_mod.potential(counts, s.L, s.M, s.N, kT, ik, chi)
    vol = float(np.float32(7.3)) ** 3
    phi = counts.astype(np.float64) / (TWO48 * (s.N / vol) * (vol / 7 ** 3))
    VA = kT * (chi[0, 0] * phi[0] + chi[0, 1] * phi[1]) + ik * (phi[0] + phi[1] - 1)
    VB = kT * (chi[1, 0] * phi[0] + chi[1, 1] * phi[1]) + ik * (phi[0] + phi[1] - 1)
    assert np.allclose(V[0], VA, rtol=1e-13, atol=1e-13)
    assert np.allclose(V[1], VB, rtol=1e-13, atol=1e-13)


def test_field_energy_derivative_is_potential(oracle_mod):
    """dW/dn_K(v) = V_K(v) with n in bead units. W is quadratic in the counts, so the
    secant slope over [n - h, n + h] equals the derivative at n exactly (up to rounding)."""
    s = wl.small_system(60, 10, 6.0, 6, K=3, n_solvent=100, seed=4)
    counts, _ = oracle_mod.density(s.R, s.T, s.L, s.M, 3)
    step = 2 ** 44                                      # 1/16 bead
    rng = np.random.default_rng(0)
    for _ in range(12):
        k, z, y, x = (rng.integers(0, 3), *rng.integers(0, 6, 3))
        mid = counts.copy()
        mid[k, z, y, x] += np.uint64(step)              # keeps mid - step >= 0
        cp, cm = mid.copy(), mid.copy()
        cp[k, z, y, x] += np.uint64(step)
        cm[k, z, y, x] -= np.uint64(step)
        V, _ = oracle_mod.potential(mid, s.L, s.M, s.N, s.kT, s.inv_kappa, s.chi)
        _, Wp = oracle_mod.potential(cp, s.L, s.M, s.N, s.kT, s.inv_kappa, s.chi)
        _, Wm = oracle_mod.potential(cm, s.L, s.M, s.N, s.kT, s.inv_kappa, s.chi)
        slope = (Wp - Wm) / (2 * step / TWO48)
        assert slope == pytest.approx(V[k, z, y, x], rel=1e-8, abs=1e-8)


# ---------------------------------------------------------------- O6-O7 ----

def test_linear_potential_exact_gradient_and_force(oracle_mod):
    """V = a.x_vertex gives g = a exactly away from the seam, and F = -a there."""
    L, M = 8.0, 16                                     # h = 1/2, powers of two
    a = np.array([0.75, -1.25, 2.5])
    h = L / M
    z, y, x = np.meshgrid(np.arange(M), np.arange(M), np.arange(M), indexing="ij")
    V = (a[0] * x * h + a[1] * y * h + a[2] * z * h)[None]
    G = oracle_mod.gradient(V, L, M)
    inner = (slice(1, M - 1),) * 3
    for d in range(3):
        assert np.all(G[0][inner][..., d] == a[d])
    rng = np.random.default_rng(1)
    xyz = 1.0 + rng.random((500, 3)) * (L - 2.6)      # cells 2..12: stencil avoids the seam
    F = oracle_mod.gather(_pos4(xyz), np.zeros(500, np.uint8), L, M, G)
    assert np.all(F == -a)


def test_lone_bead_has_no_self_force(oracle_mod):
    for seed in range(5):
        rng = np.random.default_rng(seed)
        xyz = rng.random((1, 3)) * 5.3
        s = wl.System("lone", _pos4(xyz), _pos4(np.zeros((1, 3))), np.zeros(1, np.uint8),
                      np.zeros(1, np.int32), np.full((2, 1), -1, np.int32), (5.3,) * 3,
                      (5,) * 3, 2, 1.0, 10.0, np.array([[0, 1.0], [1.0, 0]]), 100.0, 0.0, 0.03)
        Ff, _, _ = oracle_mod.forces(s)
        assert np.abs(Ff).max() < 1e-12


@pytest.mark.parametrize("n", [1, 2, 3])
def test_brute_force_pair_sum(oracle_mod, n):
    rng = np.random.default_rng(20 + n)
    L, M = (4.7, 5.9, 5.3), (5, 6, 5)
    xyz = rng.random((n, 3)) * np.array(L)
    T = rng.integers(0, 2, n).astype(np.uint8)
    chi = np.array([[0.2, 1.4], [1.4, 0.0]])
    s = wl.System("bf", _pos4(xyz), _pos4(np.zeros((n, 3))), T, np.arange(n, dtype=np.int32),
                  np.full((2, n), -1, np.int32), L, M, 2, 1.1, 6.0, chi, 0.0, 0.0, 0.03)
    Ff, _, _ = oracle_mod.forces(s)
    Fbf = bf.pair_field_forces(s.R[:, :3].astype(np.float64), T, L, M, 1.1, 6.0, chi)
    tol = 1e-12 * max(np.abs(Fbf).max(), 1.0)        # a lone bead's force is ~0
    assert np.abs(Ff - Fbf).max() <= tol
    assert np.abs(Ff.sum(0)).max() <= tol


def test_field_momentum_conservation(oracle_mod):
    s = wl.build(wl.SPECS["c1"])
    Ff, Fb, _ = oracle_mod.forces(s)
    assert np.abs(Ff.sum(0)).max() < 1e-9 * np.abs(Ff).max() * np.sqrt(s.N)
    assert np.abs(Fb.sum(0)).max() < 1e-9 * np.abs(Fb).max() * np.sqrt(s.N)


def test_chi_after_gradient_equals_gradient_after_chi(oracle_mod):
    """Algorithm 1 Kernel 4 applies chi to per-species density gradients per bead; by
    linearity of eq. 6 that equals interpolating the gradient of V (our order)."""
    s = wl.small_system(100, 10, 8.3, 8, K=3, n_solvent=200, seed=6)
    counts, _ = oracle_mod.density(s.R, s.T, s.L, s.M, 3)
    V, _ = oracle_mod.potential(counts, s.L, s.M, s.N, s.kT, s.inv_kappa, s.chi)
    F_ours = oracle_mod.gather(s.R, s.T, s.L, s.M, oracle_mod.gradient(V, s.L, s.M))
    vol = float(np.float32(8.3)) ** 3
    phi = counts.astype(np.float64) / (TWO48 * s.N / 8 ** 3)
    Gphi = oracle_mod.gradient(phi, s.L, s.M)           # d phi_K' / dr at vertices
    A = s.kT * s.chi + s.inv_kappa
    F_paper = np.zeros_like(F_ours)
    for k in range(3):
        sel = s.T == k
        Gk = np.tensordot(A[k], Gphi, axes=(0, 0))[None]
        F_paper[sel] = oracle_mod.gather(s.R[sel], np.zeros(sel.sum(), np.uint8), s.L, s.M, Gk)
    del vol
    assert np.abs(F_ours - F_paper).max() <= 1e-13 * np.abs(F_ours).max()


# ---------------------------------------------------------------- O8 -------

def test_single_bond_closed_form(oracle_mod):
    rng = np.random.default_rng(3)
    L = 10.0
    for r0 in (0.0, 0.5):
        for trial in range(20):
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            r = 0.2 + 1.5 * rng.random()
            xi = rng.random(3) * L
            if trial % 2:
                xi[0] = 0.05                           # bond crosses the x seam
                u[0] = -abs(u[0])
            xj = np.mod(xi + r * u, L)
            R = _pos4([xi, xj])
            d = R[1, :3].astype(np.float64) - R[0, :3]
            d -= L * np.rint(d / L)
            rr = np.linalg.norm(d)
            F, E = oracle_mod.bonds(R, np.array([[-1, 0], [1, -1]], np.int32), 100.0, r0, L)
            assert np.allclose(F[0], 2 * 100.0 * (rr - r0) * d / rr, rtol=1e-13, atol=1e-12)
            assert np.array_equal(F[1], -F[0])
            assert E == pytest.approx(100.0 * (rr - r0) ** 2, rel=1e-13)


def test_three_bead_chain_by_hand(oracle_mod):
    R = _pos4([[1.0, 1.0, 1.0], [2.0, 1.0, 1.0], [2.0, 3.0, 1.0]])
    bonds = np.array([[-1, 0, 1], [1, 2, -1]], np.int32)
    F, E = oracle_mod.bonds(R, bonds, 10.0, 0.0, 20.0)
    # U = 10 r^2 per bond: r01 = 1, r12 = 2 -> E = 10 + 40
    assert E == 50.0
    assert np.array_equal(F, np.array([[20.0, 0, 0], [-20.0, 40.0, 0], [0, -40.0, 0]]))


# ---------------------------------------------------------------- O9 -------

def test_harmonic_dimer_follows_exact_verlet_recurrence(oracle_mod):
    """Bonds only (chi = 0, 1/kappa = 0): the bond vector follows the closed-form VV map."""
    k, dt, n = 100.0, 0.03, 1000
    L = 64.0
    d0 = np.array([0.75, 0.0, 0.0])
    u0 = np.array([0.5, 0.0, 0.0])
    R = _pos4([[32.0, 32.0, 32.0], [32.75, 32.0, 32.0]])
    Vv = _pos4([[-0.25, 0.0, 0.0], [0.25, 0.0, 0.0]])
    s = wl.System("dimer", R, Vv, np.zeros(2, np.uint8), np.arange(2, dtype=np.int32),
                  np.array([[-1, 0], [1, -1]], np.int32), (L,) * 3, (8,) * 3, 2, 1.0, 0.0,
                  np.zeros((2, 2)), k, 0.0, dt)
    Rn, Vn, E = oracle_mod.run(s, n)
    x_exact, v_exact = bf.dimer_closed_form(d0[0], u0[0], 4 * k, dt, n)
    assert (Rn[1, 0] - Rn[0, 0]) == pytest.approx(x_exact, rel=1e-10, abs=1e-10)
    assert (Vn[1, 0] - Vn[0, 0]) == pytest.approx(v_exact, rel=1e-10, abs=1e-10)
    assert np.allclose(Rn[:, 1:], 32.0) and np.allclose(Vn.sum(0), 0.0, atol=1e-12)


def test_verlet_kinematics_and_wrap(oracle_mod):
    R = np.array([[1.0, 2.0, 3.0], [9.9, 0.05, 5.0]])
    V = np.array([[1.0, -2.0, 0.5], [4.0, -3.0, 0.0]])
    F = np.array([[2.0, 0.0, -4.0], [0.0, 0.0, 0.0]])
    dt, L = 0.1, 10.0
    R1, V1 = oracle_mod.verlet_half1(R, V, F, dt, L)
    v_half = V + 0.5 * dt * F
    assert np.allclose(V1, v_half, rtol=0, atol=1e-15)
    assert np.allclose(R1, np.mod(R + dt * v_half, L), rtol=0, atol=1e-14)
    assert np.all((R1 >= 0) & (R1 < L))
    V2, out = oracle_mod.verlet_half2(V1, F, dt)
    assert np.allclose(V2, V + dt * F, rtol=0, atol=1e-15)
    assert out[0] == pytest.approx(0.5 * (V2 ** 2).sum(), rel=1e-15)
    assert np.allclose(out[1:], V2.sum(0), atol=1e-15)
    # tiny negative coordinate wraps to 0 rather than to L
    R3, _ = oracle_mod.verlet_half1(np.array([[0.0, 1.0, 1.0]]), np.array([[-1e-300, 0, 0]]),
                                    np.zeros((1, 3)), 1.0, L)
    assert R3[0, 0] == 0.0


# ---------------------------------------------------------------- a0 -------

def test_sort_permutation_orders_by_brick_then_tag(oracle_mod):
    s = wl.small_system(300, 10, (13.1, 9.7, 21.0), (13, 10, 21), seed=9)
    sp, _ = wl.permuted(s)
    B = 4
    perm, keys = oracle_mod.sort_perm(sp.R, sp.tag, sp.L, sp.M, B)
    assert sorted(perm.tolist()) == list(range(sp.N))
    k_sorted = keys[perm]
    t_sorted = sp.tag[perm]
    order_ok = (k_sorted[:-1] < k_sorted[1:]) | ((k_sorted[:-1] == k_sorted[1:]) &
                                                   (t_sorted[:-1] < t_sorted[1:]))
    assert order_ok.all()
    nb = [(m + B - 1) // B for m in sp.M]
    for i in range(0, sp.N, 37):
        c = [bf.cell_weights(float(sp.R[i, d]), sp.L[d], sp.M[d])[0] for d in range(3)]
        brick = ((c[2] // B) * nb[1] + c[1] // B) * nb[0] + c[0] // B
        assert keys[i] == brick


# ---- O11: field-update interval (MD-SCF section; Fig. 5 refreshes the field every 300 steps)

def test_run_interval_of_one_is_run(oracle_mod):
    """A field rebuilt at every force evaluation is the plain run (or_run, a separate loop)."""
    s = wl.small_system(30, 10, 10.0, 10, seed=81)
    R1, V1, E1 = oracle_mod.run(s, 6)
    R2, V2, E2 = oracle_mod.run_interval(s, 6, 1)
    assert np.array_equal(R1, R2) and np.array_equal(V1, V2) and np.array_equal(E1, E2)


def test_run_interval_without_field_is_run(oracle_mod):
    """chi = 0 and 1/kappa = 0: V and its gradient vanish everywhere, so the rebuild schedule
    cannot change the trajectory, and W = 0."""
    s = wl.small_system(30, 10, 10.0, 10, seed=82, chi_ab=0.0, inv_kappa=0.0)
    R1, V1, E1 = oracle_mod.run(s, 6)
    for n in (2, 4, 7):
        R2, V2, E2 = oracle_mod.run_interval(s, 6, n)
        assert np.array_equal(R1, R2) and np.array_equal(V1, V2) and np.array_equal(E1, E2)
        assert not E2[:, 2].any()


def test_run_interval_schedule_from_pinned_pieces(oracle_mod):
    """Interval 3 over 7 steps composed by hand from the separately pinned density, potential,
    gradient, gather, bond and Verlet pieces: the field is rebuilt at evaluations 0, 3 and 6
    only; the others gather from the last rebuild's gradient at the current positions, and
    the reported W is the last rebuild's."""
    s = wl.small_system(30, 10, 10.0, 10, seed=83)
    n, steps = 3, 7

    def field(R):
        counts, _ = oracle_mod.density(R, s.T, s.L, s.M, s.K)
        Vp, W = oracle_mod.potential(counts, s.L, s.M, s.N, s.kT, s.inv_kappa, s.chi)
        return oracle_mod.gradient(Vp, s.L, s.M), W

    def force(R, G):
        Fb, Eb = oracle_mod.bonds(R, s.bonds, s.k_bond, s.r0, s.L)
        return oracle_mod.gather(R, s.T, s.L, s.M, G) + Fb, Eb

    R = s.R[:, :3].astype(np.float64)
    V = s.V[:, :3].astype(np.float64)
    G, W = field(R)
    F, Eb = force(R, G)
    Ws, Ebs, KEs = [W], [Eb], [0.5 * float((V * V).sum())]
    for step in range(1, steps + 1):
        R, V = oracle_mod.verlet_half1(R, V, F, s.dt, s.L)
        if step % n == 0:
            G, W = field(R)
        F, Eb = force(R, G)
        V, out = oracle_mod.verlet_half2(V, F, s.dt)
        Ws.append(W)
        Ebs.append(Eb)
        KEs.append(out[0])
    Ro, Vo, Eo = oracle_mod.run_interval(s, steps, n)
    assert np.array_equal(Ro, R) and np.array_equal(Vo, V)
    assert np.array_equal(Eo[:, 2], Ws) and np.array_equal(Eo[:, 1], Ebs)
    np.testing.assert_allclose(Eo[:, 0], KEs, rtol=1e-14)
    # the schedule matters: interval 3 differs from rebuilding every evaluation
    R1, _, _ = oracle_mod.run(s, steps)
    assert not np.array_equal(R1, Ro)


# ---- O12/O13: counter-based generator and Andersen thermostat (Integration methods section)

def test_philox_known_answers(oracle_mod):
    """Philox4x32-10 reproduces the generator's published known-answer vectors."""
    n = 0
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out = oracle_mod.philox4x32_10(w[0:4], w[4:6])
        assert [int(x) for x in out] == w[6:10]
        n += 1
    assert n == 3


def _thermo_system(n=200000, seed=3):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((n, 3))
    tag = rng.permutation(n).astype(np.int32)
    return V, tag


def test_andersen_zero_rate_leaves_velocities(oracle_mod):
    V, tag = _thermo_system(5000)
    V2, mask = oracle_mod.andersen(V, tag, 1.0, 0.0, 77, 5)
    assert not mask.any()
    assert np.array_equal(V2, V)


def test_andersen_collision_fraction_and_maxwell_statistics(oracle_mod):
    """p = 0.3: the colliding fraction is p within its binomial error; the new velocities
    are Maxwell at kT (mean 0, variance kT/m per component, normal quantiles, no
    correlation between components), and beads that do not collide keep theirs."""
    V, tag = _thermo_system()
    n = V.shape[0]
    kT = 2.5
    V2, mask = oracle_mod.andersen(V, tag, kT, 0.3, 12345, 17)
    hit = mask.astype(bool)
    frac = hit.mean()
    assert abs(frac - 0.3) <= 4.0 * np.sqrt(0.3 * 0.7 / n)
    assert np.array_equal(V2[~hit], V[~hit])
    g = V2[hit] / np.sqrt(kT)
    m = g.size
    assert abs(g.mean()) <= 4.0 / np.sqrt(m)
    assert abs(g.var() - 1.0) <= 4.0 * np.sqrt(2.0 / m)
    # fourth moment of a normal deviate is 3
    assert abs((g ** 4).mean() - 3.0) <= 4.0 * np.sqrt(96.0 / m)
    for a in range(3):
        for b in range(a + 1, 3):
            assert abs(np.mean(g[:, a] * g[:, b])) <= 4.0 / np.sqrt(g.shape[0])
    # quantiles of the standard normal
    from scipy import stats
    assert stats.kstest(g.ravel(), "norm").pvalue > 1e-4


def test_andersen_full_rate_and_mass_scaling(oracle_mod):
    """p = 1 replaces every velocity; with inverse mass 4 the deviates are scaled by
    sqrt(kT / m) = 2 sqrt(kT), bead for bead the same draws."""
    V, tag = _thermo_system(20000)
    V1, mask = oracle_mod.andersen(V, tag, 1.0, 1.0, 9, 3)
    assert mask.all()
    V4, _ = oracle_mod.andersen(V, tag, 1.0, 1.0, 9, 3, inv_mass=np.full(V.shape[0], 4.0))
    np.testing.assert_allclose(V4, 2.0 * V1, rtol=0, atol=0)
    assert abs(V1.var() - 1.0) <= 4.0 * np.sqrt(2.0 / V1.size)


def test_andersen_draws_follow_tags_not_storage(oracle_mod):
    """Draws are keyed on (tag, step): a permuted storage order permutes the result; another
    step or seed gives uncorrelated draws."""
    V, tag = _thermo_system(20000)
    Va, ma = oracle_mod.andersen(V, tag, 1.0, 0.5, 4, 8)
    perm = np.random.default_rng(1).permutation(V.shape[0])
    Vb, mb = oracle_mod.andersen(V[perm], tag[perm], 1.0, 0.5, 4, 8)
    assert np.array_equal(Vb, Va[perm]) and np.array_equal(mb, ma[perm])
    Vc, _ = oracle_mod.andersen(V, tag, 1.0, 1.0, 4, 9)
    Vd, _ = oracle_mod.andersen(V, tag, 1.0, 1.0, 5, 8)
    Ve, _ = oracle_mod.andersen(V, tag, 1.0, 1.0, 4, 8)
    for X in (Vc, Vd):
        assert abs(np.corrcoef(X.ravel(), Ve.ravel())[0, 1]) <= 4.0 / np.sqrt(X.size)


def test_run_nvt_without_collisions_is_run_interval(oracle_mod):
    s = wl.small_system(60, 10, 9.0, 9, seed=11)
    for n_f in (1, 3):
        Ra, Va, Ea = oracle_mod.run_interval(s, 12, n_f)
        Rb, Vb, Eb = oracle_mod.run_nvt(s, 12, n_f, 1.0, 0.0, 5)
        assert np.array_equal(Ra, Rb) and np.array_equal(Va, Vb) and np.array_equal(Ea, Eb)


def test_run_nvt_holds_the_bath_temperature(oracle_mod):
    """Equipartition under the thermostat: with soft bonds (k = 10) and dt = 0.01, so that
    velocity Verlet's own bias (of order (omega dt / 2)^2 for the stiffest bond mode) is
    below 0.2 %, the mean kinetic energy after equilibration is 3/2 N kT within 2 % without
    a field and within 3 % with one (the interpolated field force is not exactly
    conservative). NVE from the same start stays far hotter."""
    import dataclasses
    base = wl.small_system(200, 10, 9.0, 9, seed=12)
    soft = dataclasses.replace(base, k_bond=10.0, dt=0.01)
    free = dataclasses.replace(soft, inv_kappa=0.0, chi=np.zeros((2, 2)))
    for sysm, tol in ((free, 0.02), (soft, 0.03)):
        _, _, E = oracle_mod.run_nvt(sysm, 1000, 1, 1.0, 0.1, 2024)
        ke = E[500:, 0].mean() / sysm.N
        assert abs(ke - 1.5) <= tol * 1.5, (tol, ke)
    _, _, E0 = oracle_mod.run(base, 100)
    assert E0[50:, 0].mean() / base.N > 10.0


# ---- O7P: the paper-literal staggered gather (reading P of Algorithm 1 Kernels 3-4)

def _beads_away_from_seam(rng, n, L, M, margin=2.0):
    h = L / M
    R = np.zeros((n, 4), np.float32)
    R[:, :3] = rng.uniform(margin * h, L - margin * h, (n, 3)).astype(np.float32)
    return R


def test_staggered_uniform_field_gives_no_force(oracle_mod):
    rng = np.random.default_rng(1)
    L, M = 16.0, 16
    R = _beads_away_from_seam(rng, 500, L, M, margin=0.0)
    T = rng.integers(0, 2, 500).astype(np.uint8)
    Phi = np.full((2, M, M, M), 0.731)
    A = np.array([[0.3, 1.7], [1.7, -0.4]])
    F = oracle_mod.gather_staggered(R, T, L, M, Phi, A)
    assert np.array_equal(F, np.zeros_like(F))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_staggered_quadratic_potential_gives_exact_linear_force(oracle_mod, axis):
    """V = x_d^2 at the vertices: the blend of the backward and forward differences at the
    nearest vertex, weighted 1/2 - delta and 1/2 + delta, is exactly -dV/dx_d = -2 x_d at the
    (quantised) bead position, for beads whose stencil avoids the periodic seam; the other
    components vanish. Swapped or shifted fraction ratios would not be exact."""
    rng = np.random.default_rng(2 + axis)
    L, M = 16.0, 16                      # h = 1: vertex coordinates are exact
    R = _beads_away_from_seam(rng, 400, L, M)
    T = np.zeros(400, np.uint8)
    x = np.arange(M, dtype=np.float64)
    shape = [1, 1, 1]
    shape[2 - axis] = M
    Phi = np.broadcast_to((x ** 2).reshape(shape), (M, M, M))[None].copy()
    F = oracle_mod.gather_staggered(R, T, L, M, Phi, np.eye(1))
    u = R[:, axis].astype(np.float64)
    q = np.floor((u - np.floor(u)) * 65536.0)
    xq = np.floor(u) + q / 65536.0           # the position the weights see
    np.testing.assert_array_equal(F[:, axis], -2.0 * xq)
    others = [d for d in range(3) if d != axis]
    assert not F[:, others].any()


def test_staggered_linear_potential_exact_and_midpoint_continuity(oracle_mod):
    """V = a x (a = 0.25, h = 0.5): F = -a exactly; a bead exactly half-way between two
    vertices takes the forward difference at the lower vertex, the same value as the backward
    difference at the upper one."""
    L, M, a = 8.0, 16, 0.25
    h = L / M
    x = np.arange(M) * h
    Phi = np.broadcast_to((a * x).reshape(1, 1, M), (M, M, M))[None].copy()
    R = np.array([[3.0 + 0.5 * h, 4.0, 4.0, 0.0], [3.1, 3.7, 4.9, 0.0]], np.float32)
    F = oracle_mod.gather_staggered(R, np.zeros(2, np.uint8), L, M, Phi, np.eye(1))
    np.testing.assert_array_equal(F[:, 0], [-a, -a])
    assert not F[:, 1:].any()


def test_staggered_paper_order_equals_potential_first(oracle_mod):
    """Kernel 4's order (differences of phi per species, then kT chi + 1/kappa) equals the
    differences of V with unit coefficients, to rounding (eq. 6 is linear)."""
    s = wl.small_system(300, 10, 11.0, 11, K=3, n_solvent=2000, seed=31)
    counts, _ = oracle_mod.density(s.R, s.T, s.L, s.M, s.K)
    V, _ = oracle_mod.potential(counts, s.L, s.M, s.N, s.kT, s.inv_kappa, s.chi)
    vol = float(np.prod(np.asarray(s.L, dtype=np.float32).astype(np.float64)))
    nm = int(np.prod(s.M))
    phi = counts.astype(np.float64) / (2.0 ** 48 * (s.N / vol) * (vol / nm))
    A = s.kT * np.asarray(s.chi) + s.inv_kappa
    Fp = oracle_mod.gather_staggered(s.R, s.T, s.L, s.M, phi, A)
    Fv = oracle_mod.gather_staggered(s.R, s.T, s.L, s.M, V, np.eye(s.K))
    assert np.abs(Fp - Fv).max() <= 1e-12 * np.abs(Fv).max()
    # each bead feels only its own species' row of A
    Fr = oracle_mod.gather_staggered(s.R, s.T, s.L, s.M, V, np.diag([1.0, 0.0, 0.0]))
    assert not Fr[s.T != 0].any() and np.array_equal(Fr[s.T == 0], Fv[s.T == 0])


# ---- O8A: angle potentials (Bonded forces section)

def _angle_table_for(triplets, N):
    """Per-bead angle table [3A, N] (partner, partner, role) of a list of (end, middle, end)."""
    rows = {}
    for (i, j, k) in triplets:
        for bead, entry in ((i, (j, k, 0)), (j, (i, k, 1)), (k, (j, i, 0))):
            rows.setdefault(bead, []).append(entry)
    A = max((len(v) for v in rows.values()), default=0)
    tab = np.full((3 * A, N), -1, np.int32)
    for bead, entries in rows.items():
        for a, (p, q, role) in enumerate(entries):
            tab[3 * a, bead], tab[3 * a + 1, bead], tab[3 * a + 2, bead] = p, q, role
    tab[2::3][tab[0::3] < 0] = 0
    return tab


def test_angle_right_triplet_by_hand(oracle_mod):
    """Ends at (1,0,0) and (0,1,0), middle at the origin: theta = pi/2. Cosine form with
    theta0 = 2 pi / 3 (cos theta0 = -1/2), k = 3: U = 3 (0 + 1/2)^2 = 3/4; dU/dcos = 3, and
    d cos/d x_end1 = (0,1,0), d cos/d x_end2 = (1,0,0), so F_end1 = (0,-3,0),
    F_end2 = (-3,0,0), F_mid = (3,3,0): the ends are pushed apart, opening the angle.
    Harmonic form with theta0 = pi/3: U = k (pi/6)^2, dU/dtheta = k pi / 3 and
    |d theta / d x_end| = 1 / |a| = 1, so F_end1 = (0, k pi/3, 0) closes the angle."""
    L = (10.0, 10.0, 10.0)
    R = np.array([[6.0, 5.0, 5.0], [5.0, 5.0, 5.0], [5.0, 6.0, 5.0]])
    tab = _angle_table_for([(0, 1, 2)], 3)
    F, E = oracle_mod.angles(R, tab, 3.0, 2.0 * np.pi / 3.0, 1, L)
    np.testing.assert_allclose(F, [[0.0, -3.0, 0.0], [3.0, 3.0, 0.0], [-3.0, 0.0, 0.0]], atol=1e-14)
    assert E == pytest.approx(0.75, rel=1e-14)
    k = 2.0
    F, E = oracle_mod.angles(R, tab, k, np.pi / 3.0, 0, L)
    np.testing.assert_allclose(F[0], [0.0, k * np.pi / 3.0, 0.0], atol=1e-13)
    np.testing.assert_allclose(F[2], [k * np.pi / 3.0, 0.0, 0.0], atol=1e-13)
    assert E == pytest.approx(k * (np.pi / 6.0) ** 2, rel=1e-14)


@pytest.mark.parametrize("form", [0, 1])
def test_angle_forces_are_minus_the_energy_gradient(oracle_mod, form):
    """Random bent chains across the periodic seam: every force component equals the central
    finite difference of the angle energy, and the forces sum to zero."""
    rng = np.random.default_rng(7 + form)
    L = (6.0, 7.0, 5.5)
    n_chain, length = 12, 6
    R = []
    for c in range(n_chain):
        x = rng.uniform(0, 1, 3) * np.asarray(L)
        for b in range(length):
            R.append(x.copy())
            x = x + rng.normal(0, 0.6, 3)
    R = np.mod(np.asarray(R), np.asarray(L))
    N = len(R)
    trip = [(c * length + b, c * length + b + 1, c * length + b + 2)
            for c in range(n_chain) for b in range(length - 2)]
    tab = _angle_table_for(trip, N)
    k, th0 = 4.0, 1.9
    F, E = oracle_mod.angles(R, tab, k, th0, form, L)
    eps = 1e-6
    Fd = np.zeros_like(F)
    for i in range(N):
        for d in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[i, d] += eps
            Rm[i, d] -= eps
            Fd[i, d] = -(oracle_mod.angles(Rp, tab, k, th0, form, L)[1] -
                         oracle_mod.angles(Rm, tab, k, th0, form, L)[1]) / (2 * eps)
    assert np.abs(F - Fd).max() <= 1e-6 * np.abs(F).max()
    assert np.abs(F.sum(0)).max() <= 1e-10 * np.abs(F).max()
    # the energy is that of each angle once, whichever member evaluates it
    th = []
    for (i, j, kk) in trip:
        a = R[i] - R[j]
        b = R[kk] - R[j]
        a -= np.asarray(L) * np.rint(a / np.asarray(L))
        b -= np.asarray(L) * np.rint(b / np.asarray(L))
        th.append(np.arccos(np.dot(a, b) / np.linalg.norm(a) / np.linalg.norm(b)))
    th = np.asarray(th)
    want = (k * (th - th0) ** 2).sum() if form == 0 else (k * (np.cos(th) - np.cos(th0)) ** 2).sum()
    assert E == pytest.approx(want, rel=1e-9)


def test_angle_energy_invariant_under_rotation(oracle_mod):
    rng = np.random.default_rng(3)
    R = rng.uniform(20, 30, (3, 3))
    L = (100.0, 100.0, 100.0)
    tab = _angle_table_for([(0, 1, 2)], 3)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    R2 = (R - 25.0) @ q.T + 50.0
    for form in (0, 1):
        F1, E1 = oracle_mod.angles(R, tab, 1.5, 2.0, form, L)
        F2, E2 = oracle_mod.angles(R2, tab, 1.5, 2.0, form, L)
        assert E2 == pytest.approx(E1, rel=1e-12)
        np.testing.assert_allclose(F2, F1 @ q.T, atol=1e-12 * np.abs(F1).max())


def test_angle_types_select_their_parameters(oracle_mod):
    """A table holding a harmonic triplet (type 0) and a cosine triplet (type 1) gives the sum
    of the two evaluated alone with their own parameters."""
    rng = np.random.default_rng(9)
    L = (20.0, 20.0, 20.0)
    R = rng.uniform(5, 8, (6, 3))
    both = _angle_table_for([(0, 1, 2), (3, 4, 5)], 6)
    both[2::3][both[0::3] >= 0] += 2 * (np.arange(6) >= 3)[None, :].repeat(both.shape[0] // 3, 0)[
        both[0::3] >= 0]
    Fa, Ea = oracle_mod.angles(R, _angle_table_for([(0, 1, 2)], 6), 2.0, 1.1, 0, L)
    Fb, Eb = oracle_mod.angles(R, _angle_table_for([(3, 4, 5)], 6), 5.0, 2.9, 1, L)
    F, E = oracle_mod.angles(R, both, [2.0, 5.0], [1.1, 2.9], [0, 1], L)
    np.testing.assert_allclose(F, Fa + Fb, rtol=0, atol=1e-14 * np.abs(F).max())
    assert E == pytest.approx(Ea + Eb, rel=1e-14)
