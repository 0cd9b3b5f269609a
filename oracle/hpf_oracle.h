/*
 * FP64 CPU oracle of the hybrid particle-field MD (MD-SCF / hPF-MD) timestep.
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow, obviously-correct
 * reference that the HIP path is checked against. Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does. It shares no code, header, table or helper with
 * the HIP library.
 *
 * Every floating-point quantity is computed in double precision. The one
 * place where floating point decides an integer -- the cell coordinate
 * u = x * s that picks a bead's cell and its fixed-point cloud-in-cell
 * weights -- is taken in FP32 (one IEEE single rounding of the exact
 * product), because that quantisation is part of the method's encoding and
 * both sides must take the same integer decision.
 *
 * Paper: Zhu et al., "GALAMOST: GPU-accelerated large-scale molecular
 * simulation toolkit" (arXiv 1310.2041), section "The MD-SCF treatment of
 * interparticle forces", eqs. (4)-(6), Algorithm 1; section "Bonded forces",
 * eq. (7); section "Integration methods" (velocity Verlet, periodic box).
 *
 * Parity status per function is listed in the header comment of each
 * function in hpf_oracle.c.
 */
#ifndef HPF_ORACLE_H
#define HPF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_FIX_BITS 16                 /* S: bits of the 1-D fixed-point weight */
#define OR_ONE (1u << OR_FIX_BITS)     /* 2^S */
#define OR_MAX_TYPES 8

typedef struct {
    double L[3];   /* box edges (the FP32 box widened to double) */
    int32_t M[3];  /* mesh points = cells per edge (periodic) */
    float s[3];    /* quantisation scale, fl32(M / L) */
} or_mesh_t;

/* Fill a mesh description from the FP32 box edges and the mesh size. */
void or_mesh_init(or_mesh_t* m, const float L[3], const int32_t M[3]);

/* O1-O2 for one coordinate: cell index c (mod M) and the two 1-D weights
 * w[0] = 2^S - q (lower vertex), w[1] = q (upper vertex). Returns 0, or 1
 * when the coordinate is not finite or |x*s| >= 2^24 (bead skipped). */
int or_cell_weights(double x, float s, int32_t M, int32_t* c, uint32_t w[2]);

/* O3: counts[K][Mz][My][Mx] += fixed-point CIC weights of every bead.
 * R is double [N][3]. Returns the number of skipped (invalid) beads. */
int64_t or_density(const double* R, const uint8_t* T, int64_t N, const or_mesh_t* m,
                   int32_t K, uint64_t* counts);

/* O4-O5 and O10(W): potential V[K][M^3] from the counts (eq. 4), plus the
 * field energy W if W != NULL. n_beads is the total bead count that fixes
 * the mean density rho0 = N / V_box. */
void or_potential(const uint64_t* counts, const or_mesh_t* m, int64_t n_beads, int32_t K,
                  double kT, double inv_kappa, const double* chi, double* V, double* W);

/* O6: centred periodic gradient G[K][M^3][3] of V. */
void or_gradient(const double* V, const or_mesh_t* m, int32_t K, double* G);

/* O7: field force F[N][3] = -sum_a (W_a / 2^3S) G_{T_i}(c_i + a) (overwrites F). */
int64_t or_gather(const double* R, const uint8_t* T, int64_t N, const or_mesh_t* m,
                  int32_t K, const double* G, double* F);

/* O8: harmonic bonds U = k (r - r0)^2 (eq. 7); F[N][3] += ; *E (if non-NULL)
 * receives the bond energy, every bond counted once. bonds is the table
 * [D][N] of partner indices (-1 = none). */
void or_bonds(const double* R, int64_t N, const int32_t* bonds, int32_t D, double k,
              double r0, const double L[3], double* F, double* E);

/* O8A angles (Bonded forces section): the angle theta at the middle bead j of
 * a triplet (i, j, k) between the minimum-image vectors a = x_i - x_j and
 * b = x_k - x_j, cos(theta) = a.b / (|a| |b|), theta = atan2(|a x b|, a.b).
 *   form 0 (harmonic):  U = k (theta - theta0)^2
 *   form 1 (cosine):    U = k (cos(theta) - cos(theta0))^2
 * Stored as the bonds are, per bead: angles[(3a + 0) N + i] and
 * angles[(3a + 1) N + i] are the other two members of the bead's a-th angle and
 * code = angles[(3a + 2) N + i] = role + 2 type: role 1 if the bead is the
 * middle, 0 if it is an end (the first partner then being the middle); type
 * selects k[type], theta0[type], form[type] (type < ntypes). A first partner
 * < 0 means no angle.
 * Each angle is evaluated from each of its three members, every member taking
 * its own force -dU/dx; *E (if non-NULL) receives the angle energy, each angle
 * counted once. For the harmonic form dU/dcos = -2k (theta - theta0) / sin(theta),
 * with sin(theta) floored at 1e-3 (reading: the force of an exactly straight
 * triplet is otherwise undefined). F[N][3] is accumulated. */
void or_angles(const double* R, int64_t N, const int32_t* angles, int32_t A, int32_t ntypes,
               const double* k, const double* theta0, const int32_t* form, const double L[3], double* F,
               double* E);

/* O9: first half of velocity Verlet: v += dt/2 F/m; x += dt v; wrap to [0, L). */
void or_verlet_half1(double* R, double* V, const double* F, const double* inv_mass,
                     int64_t N, double dt, const double L[3]);
/* O9: second half: v += dt/2 F/m. out4 (if non-NULL) = {KE, Px, Py, Pz}. */
void or_verlet_half2(double* V, const double* F, const double* inv_mass, int64_t N,
                     double dt, double* out4);

/* Full force evaluation (O1-O8). F is overwritten; energies (nullable)
 * receive {W, E_bond}. Work arrays are allocated internally. Returns the
 * number of skipped beads, or -1 on allocation failure. */
typedef struct {
    const or_mesh_t* mesh;
    int32_t K;
    double kT, inv_kappa;
    const double* chi;      /* [K][K] */
    const int32_t* bonds;   /* [D][N] */
    int32_t D;
    double k_bond, r0;
} or_params_t;

int64_t or_forces(const double* R, const uint8_t* T, int64_t N, const or_params_t* p,
                  double* F_field, double* F_bond, double* energies2);

/* n_steps of velocity Verlet from (R, V). energies [n_steps+1][4] receives
 * {KE, E_bond, W, E_tot} at the start and after every step. inv_mass may be
 * NULL (unit masses). Returns 0, or -1 on allocation failure. */
int or_run(double* R, double* V, const uint8_t* T, const double* inv_mass, int64_t N,
           const or_params_t* p, double dt, int32_t n_steps, double* energies);

/* or_run with the density field rebuilt only at every field_every-th force
 * evaluation (O11): evaluation s (0 at the start, s after step s) rebuilds
 * n_K, V and G when s % field_every == 0; the others gather from the last G.
 * energies as in or_run, W being that of the last rebuild. field_every = 1
 * is or_run. Returns 0, -1 on allocation failure, -2 for field_every < 1. */
int or_run_interval(double* R, double* V, const uint8_t* T, const double* inv_mass, int64_t N,
                    const or_params_t* p, double dt, int32_t n_steps, int32_t field_every,
                    double* energies);

/* O7P staggered gather (reading P of Algorithm 1 Kernels 3-4): per axis d the
 * bead's nearest vertex n_d (u_d = fl32(x_d s_d), quantised fraction q_d/2^S as
 * in O2: n_d = c_d when q_d < 2^(S-1), else c_d + 1) and delta_d = u_d - n_d
 * (quantised, in [-1/2, 1/2)); the backward and forward differences of each
 * field Phi_K' at n along d (Kernel 3), blended with the fraction ratios
 * 1/2 - delta_d and 1/2 + delta_d and summed with the coefficients
 * A[T_i][K'] (Kernel 4):
 *   F_i,d = -(1/h_d) sum_K' A[T_i][K'] ((1/2 - delta_d)(Phi_K'(n) - Phi_K'(n - e_d))
 *                                     + (1/2 + delta_d)(Phi_K'(n + e_d) - Phi_K'(n))).
 * With Phi = phi and A = kT chi + 1/kappa this is the paper's order; with Phi = V
 * and A = identity it is the same force (eq. 6 is linear). Phi is [K][M^3];
 * A is [K][K]. Returns the number of skipped beads (F = 0 for them). */
int64_t or_gather_staggered(const double* R, const uint8_t* T, int64_t N, const or_mesh_t* m,
                            int32_t K, const double* Phi, const double* A, double* F);

/* O12 counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter
 * and a 2 x 32-bit key give 4 x 32 random bits through ten rounds of two
 * 32 x 32 -> 64-bit products with Weyl-sequence key updates. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* O13 Andersen thermostat (Integration methods section: NVT by the Andersen
 * thermostat). At time level `step` bead i (tag t_i) collides with the heat
 * bath with probability p (= collision rate x dt): the 24-bit uniform
 * integer (r0 >> 8) of Philox(ctr = (t_i, step_lo, step_hi, 0), key = seed)
 * is compared with floor(p 2^24) in integers. A colliding bead gets
 * v = sqrt(kT / m) (g0, g1, g2), g from Box-Muller on the 24-bit uniforms
 * u = (r >> 8 [+ 1]) 2^-24 of r1, r2 (g0 = rad cos, g1 = rad sin) and of r3
 * and word 0 of the counter (t_i, step_lo, step_hi, 1) (g2 = rad cos).
 * Returns the number of collisions. mask (nullable) receives 1 per colliding bead. */
int64_t or_andersen(double* V, const int32_t* tag, const double* inv_mass, int64_t N, double kT,
                    float p, uint64_t seed, int64_t step, uint8_t* mask);

/* or_run_interval with the Andersen thermostat applied after the second half
 * kick of every step s (time level s), before that step's kinetic energy is
 * taken. p = 0 is or_run_interval. */
int or_run_nvt(double* R, double* V, const uint8_t* T, const int32_t* tag, const double* inv_mass,
               int64_t N, const or_params_t* p, double dt, int32_t n_steps, int32_t field_every,
               double kT, float p_coll, uint64_t seed, double* energies);

/* a0: cell-list order (the paper reorders particles for cache hits and bins
 * them into cells, Algorithm 1 Kernel 1). key = index of the brick of B^3
 * cells holding the bead's cell, bricks numbered x fastest; beads that
 * cannot be binned get key 0xFFFFFFFF. perm receives the bead order sorted
 * by (key, tag): every brick's beads are one contiguous range, in tag order.
 * keys (nullable) receives each bead's key in the input order. */
int or_sort_perm(const double* R, const int32_t* tag, int64_t N, const or_mesh_t* m,
                 int32_t B, int64_t* perm, uint32_t* keys);

#ifdef __cplusplus
}
#endif
#endif
