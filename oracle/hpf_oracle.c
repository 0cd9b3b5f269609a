/*
 * FP64 CPU oracle of the hPF-MD (MD-SCF) timestep -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain loops in the order the method defines them, no blocking, no fusion.
 * See hpf_oracle.h for the conventions. The quantities and the readings of
 * the paper they rest on:
 *
 *   O1 cell coordinate  u = fl32(x * s), s = fl32(M / L); c = floor(u) mod M;
 *                       f = fl32(u - floor(u)).
 *   O2 1-D weights      q = floor(f * 2^S); w0 = 2^S - q, w1 = q. Vertex
 *                       c + a (a in {0,1}^3, periodic) receives the product
 *                       W_a = w_ax * w_ay * w_az; sum_a W_a = 2^3S exactly.
 *                       (MD-SCF section: a bead spreads its density fractions
 *                       over the eight vertices of its cell; the number of
 *                       vertices equals the number of cells, Algorithm 1
 *                       Kernel 2, so the vertex mesh is periodic.)
 *   O3 counts           n_K(v) = sum over beads of type K of W_a  (uint64).
 *   O4 normalisation    phi_K = n_K / (2^3S rho0 dV), rho0 = N / V_box,
 *                       dV = V_box / M^3 (reading: the paper does not state it;
 *                       this choice makes a uniform melt give sum_K phi_K = 1).
 *   O5 potential        V_K = kT sum_K' chi_KK' phi_K' + (1/kappa)(sum_K phi_K - 1)
 *                       (eq. 4; eq. 5 is its two-species case).
 *   O6 gradient         g_K,d(v) = (V_K(v + e_d) - V_K(v - e_d)) / (2 h_d),
 *                       h_d = L_d / M_d, periodic (reading of Algorithm 1
 *                       Kernel 3: a centred difference at the vertex instead of
 *                       the staggered pair).
 *   O7 gather           F_i = -sum_a (W_a / 2^3S) g_{T_i}(c_i + a): the field
 *                       force of eq. 6, interpolated with the same weights used
 *                       for the density (Algorithm 1 Kernel 4, reading).
 *   O7P staggered       (or_gather_staggered) the paper-literal reading of
 *                       Algorithm 1 Kernels 3-4: staggered backward and forward
 *                       differences at the bead's nearest vertex, blended by the
 *                       fraction ratios 1/2 -+ (u - n), no transverse weights.
 *   O8 bonds            U = k (r - r0)^2 (eq. 7, no factor 1/2); d = minimum
 *                       image of x_j - x_i; F_i += 2k (r - r0) d / r.
 *   O8A angles          (or_angles) the two angle forms of the Bonded forces
 *                       section, k (theta - theta0)^2 and k (cos theta -
 *                       cos theta0)^2, theta at the middle bead; stored and
 *                       evaluated per bead like the bonds (three times per angle).
 *   O9 velocity Verlet  (Integration methods section) with unit mass by
 *                       default and wrapping into the periodic box.
 *   O10 energies        KE = sum m v^2 / 2; E_bond = sum over bonds of U;
 *                       W = rho0 dV sum_v [ kT/2 sum_KK' chi phi_K phi_K'
 *                       + 1/(2 kappa) (sum_K phi_K - 1)^2 ], the functional
 *                       whose derivative by the bead count at v is V_K(v).
 *   O12 generator       Philox4x32-10 (counter-based; or_philox4x32_10).
 *   O13 Andersen        (or_andersen, or_run_nvt) the Integration methods
 *                       section names the Andersen thermostat for NVT: after
 *                       the second half kick of step s, each bead collides
 *                       with probability p = (collision rate) dt and takes a
 *                       new velocity from the Maxwell distribution at kT;
 *                       the decision and the deviates come from O12 keyed on
 *                       (tag, s), so they do not depend on the storage order.
 *   O11 field interval  (or_run_interval) the MD-SCF section keeps the stiff
 *                       bonded terms on the small time step but rebuilds the
 *                       soft density field only after many steps (the DPPC
 *                       comparison of Fig. 5 uses 300). Force evaluation s
 *                       (s = 0 at the start, s after step s) rebuilds n_K, V
 *                       and G from the positions when s is a multiple of the
 *                       interval; in between, O7 uses the G of the last
 *                       rebuild at the current positions. Bonds are evaluated
 *                       every time. Reported W is that of the last rebuild
 *                       (reading: the field in force).
 *
 * Loops carry OpenMP pragmas that the parity build (no -fopenmp) ignores; a
 * separately compiled OpenMP build serves only to time the oracle on all host
 * cores (its density adds stay exact; its FP64 sums are regrouped by thread).
 *
 * Pins (what fixes each function independently of this file) are in the
 * CPU test suite: partition of unity, hand-derived single-bead weights,
 * uniform melt, linear potential, whole-cell translation, permutation
 * invariance, a brute-force pair-kernel evaluation for 1-3 beads, the
 * closed-form bond force, the exact velocity-Verlet recurrence of a harmonic
 * dimer, and a finite-difference check of dW/dn = V.
 */
#include "hpf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double TWO_3S = 281474976710656.0; /* 2^48 = (2^S)^3 */

void or_mesh_init(or_mesh_t* m, const float L[3], const int32_t M[3])
{
    for (int d = 0; d < 3; ++d) {
        m->L[d] = (double)L[d];
        m->M[d] = M[d];
        m->s[d] = (float)((double)M[d] / (double)L[d]);
    }
}

int or_cell_weights(double x, float s, int32_t M, int32_t* c, uint32_t w[2])
{
    if (!isfinite(x))
        return 1;
    float u = (float)(x * (double)s);          /* O1: one FP32 rounding */
    if (!(fabsf(u) < 16777216.0f))
        return 1;
    double fl = floor((double)u);
    float f = (float)((double)u - fl);         /* fractional part, FP32 */
    uint32_t q = (uint32_t)floor((double)f * (double)OR_ONE);   /* O2 */
    int64_t ci = ((int64_t)fl) % M;
    if (ci < 0)
        ci += M;
    *c = (int32_t)ci;
    w[0] = OR_ONE - q;
    w[1] = q;
    return 0;
}

/* Cell and weights of bead i in all three dimensions; 0 if valid. */
static int bead_cell(const double* R, int64_t i, const or_mesh_t* m, int32_t c[3],
                     uint32_t w[3][2])
{
    for (int d = 0; d < 3; ++d)
        if (or_cell_weights(R[3 * i + d], m->s[d], m->M[d], &c[d], w[d]))
            return 1;
    return 0;
}

static int64_t vertex_index(const or_mesh_t* m, int32_t x, int32_t y, int32_t z)
{
    return ((int64_t)z * m->M[1] + y) * m->M[0] + x;
}

int64_t or_density(const double* R, const uint8_t* T, int64_t N, const or_mesh_t* m,
                   int32_t K, uint64_t* counts)
{
    const int64_t nm = (int64_t)m->M[0] * m->M[1] * m->M[2];
    int64_t skipped = 0;
#pragma omp parallel for reduction(+ : skipped) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int32_t c[3];
        uint32_t w[3][2];
        if (T[i] >= K || bead_cell(R, i, m, c, w)) {
            ++skipped;
            continue;
        }
        uint64_t* nk = counts + (int64_t)T[i] * nm;
        for (int az = 0; az < 2; ++az)
            for (int ay = 0; ay < 2; ++ay)
                for (int ax = 0; ax < 2; ++ax) {
                    int32_t vx = (c[0] + ax) % m->M[0];
                    int32_t vy = (c[1] + ay) % m->M[1];
                    int32_t vz = (c[2] + az) % m->M[2];
                    uint64_t Wa = (uint64_t)w[0][ax] * w[1][ay] * w[2][az];
#pragma omp atomic
                    nk[vertex_index(m, vx, vy, vz)] += Wa;
                }
    }
    return skipped;
}

void or_potential(const uint64_t* counts, const or_mesh_t* m, int64_t n_beads, int32_t K,
                  double kT, double inv_kappa, const double* chi, double* V, double* W)
{
    const int64_t nm = (int64_t)m->M[0] * m->M[1] * m->M[2];
    const double vol = m->L[0] * m->L[1] * m->L[2];
    const double rho0 = (double)n_beads / vol;
    const double dV = vol / (double)nm;
    double w_sum = 0.0;
#pragma omp parallel for reduction(+ : w_sum) schedule(static)
    for (int64_t v = 0; v < nm; ++v) {
        double phi[OR_MAX_TYPES];
        double total = 0.0;
        for (int k = 0; k < K; ++k) {
            phi[k] = n_beads > 0 ? (double)counts[k * nm + v] / (TWO_3S * rho0 * dV) : 0.0;
            total += phi[k];
        }
        double delta = total - 1.0;
        double inter = 0.0;
        for (int k = 0; k < K; ++k) {
            double mix = 0.0;
            for (int kk = 0; kk < K; ++kk)
                mix += chi[k * K + kk] * phi[kk];
            V[k * nm + v] = kT * mix + inv_kappa * delta;
            inter += phi[k] * mix;
        }
        w_sum += 0.5 * kT * inter + 0.5 * inv_kappa * delta * delta;
    }
    if (W)
        *W = rho0 * dV * w_sum;
}

void or_gradient(const double* V, const or_mesh_t* m, int32_t K, double* G)
{
    const int32_t Mx = m->M[0], My = m->M[1], Mz = m->M[2];
    const int64_t nm = (int64_t)Mx * My * Mz;
    const double h[3] = {m->L[0] / Mx, m->L[1] / My, m->L[2] / Mz};
    for (int k = 0; k < K; ++k) {
        const double* Vk = V + k * nm;
#pragma omp parallel for schedule(static)
        for (int32_t z = 0; z < Mz; ++z)
            for (int32_t y = 0; y < My; ++y)
                for (int32_t x = 0; x < Mx; ++x) {
                    int64_t v = vertex_index(m, x, y, z);
                    double* g = G + 3 * (k * nm + v);
                    g[0] = (Vk[vertex_index(m, (x + 1) % Mx, y, z)] -
                            Vk[vertex_index(m, (x + Mx - 1) % Mx, y, z)]) / (2.0 * h[0]);
                    g[1] = (Vk[vertex_index(m, x, (y + 1) % My, z)] -
                            Vk[vertex_index(m, x, (y + My - 1) % My, z)]) / (2.0 * h[1]);
                    g[2] = (Vk[vertex_index(m, x, y, (z + 1) % Mz)] -
                            Vk[vertex_index(m, x, y, (z + Mz - 1) % Mz)]) / (2.0 * h[2]);
                }
    }
}

int64_t or_gather(const double* R, const uint8_t* T, int64_t N, const or_mesh_t* m,
                  int32_t K, const double* G, double* F)
{
    const int64_t nm = (int64_t)m->M[0] * m->M[1] * m->M[2];
    int64_t skipped = 0;
#pragma omp parallel for reduction(+ : skipped) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double f[3] = {0.0, 0.0, 0.0};
        int32_t c[3];
        uint32_t w[3][2];
        if (T[i] >= K || bead_cell(R, i, m, c, w)) {
            ++skipped;
        } else {
            const double* Gk = G + 3 * (int64_t)T[i] * nm;
            for (int az = 0; az < 2; ++az)
                for (int ay = 0; ay < 2; ++ay)
                    for (int ax = 0; ax < 2; ++ax) {
                        int64_t v = vertex_index(m, (c[0] + ax) % m->M[0],
                                                 (c[1] + ay) % m->M[1], (c[2] + az) % m->M[2]);
                        double Wa = (double)((uint64_t)w[0][ax] * w[1][ay] * w[2][az]) / TWO_3S;
                        for (int d = 0; d < 3; ++d)
                            f[d] -= Wa * Gk[3 * v + d];
                    }
        }
        for (int d = 0; d < 3; ++d)
            F[3 * i + d] = f[d];
    }
    return skipped;
}

/* O7P: nearest vertex and offset along one axis, from the O1-O2 quantities. */
static void nearest_vertex(int32_t c, uint32_t q, int32_t M, int32_t* n, double* delta)
{
    const uint32_t half = OR_ONE / 2;
    if (q < half) {
        *n = c;
        *delta = (double)q / (double)OR_ONE;
    } else {
        *n = (c + 1) % M;
        *delta = ((double)q - (double)OR_ONE) / (double)OR_ONE;
    }
}

int64_t or_gather_staggered(const double* R, const uint8_t* T, int64_t N, const or_mesh_t* m,
                            int32_t K, const double* Phi, const double* A, double* F)
{
    const int64_t nm = (int64_t)m->M[0] * m->M[1] * m->M[2];
    const double h[3] = {m->L[0] / m->M[0], m->L[1] / m->M[1], m->L[2] / m->M[2]};
    int64_t skipped = 0;
    for (int64_t i = 0; i < N; ++i) {
        int32_t c[3];
        uint32_t w[3][2];
        double f[3] = {0.0, 0.0, 0.0};
        if (T[i] >= K || bead_cell(R, i, m, c, w)) {
            ++skipped;
        } else {
            int32_t n[3];
            double delta[3];
            for (int d = 0; d < 3; ++d)
                nearest_vertex(c[d], w[d][1], m->M[d], &n[d], &delta[d]);
            const int64_t v0 = vertex_index(m, n[0], n[1], n[2]);
            for (int d = 0; d < 3; ++d) {
                int32_t lo[3] = {n[0], n[1], n[2]}, hi[3] = {n[0], n[1], n[2]};
                lo[d] = (n[d] + m->M[d] - 1) % m->M[d];
                hi[d] = (n[d] + 1) % m->M[d];
                const int64_t vlo = vertex_index(m, lo[0], lo[1], lo[2]);
                const int64_t vhi = vertex_index(m, hi[0], hi[1], hi[2]);
                const double xf1 = 0.5 - delta[d], xf2 = 0.5 + delta[d];
                double sum = 0.0;
                for (int kk = 0; kk < K; ++kk) {
                    const double* P = Phi + kk * nm;
                    const double g1 = P[v0] - P[vlo];       /* backward difference (Kernel 3) */
                    const double g2 = P[vhi] - P[v0];       /* forward difference */
                    sum += A[T[i] * K + kk] * (xf1 * g1 + xf2 * g2);
                }
                f[d] = -sum / h[d];
            }
        }
        for (int d = 0; d < 3; ++d)
            F[3 * i + d] = f[d];
    }
    return skipped;
}

void or_bonds(const double* R, int64_t N, const int32_t* bonds, int32_t D, double k,
              double r0, const double L[3], double* F, double* E)
{
    double e = 0.0;
#pragma omp parallel for reduction(+ : e) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        for (int32_t b = 0; b < D; ++b) {
            int32_t j = bonds[(int64_t)b * N + i];
            if (j < 0)
                continue;
            double d[3], r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                d[a] = R[3 * (int64_t)j + a] - R[3 * i + a];
                d[a] -= L[a] * nearbyint(d[a] / L[a]);    /* minimum image */
                r2 += d[a] * d[a];
            }
            double r = sqrt(r2);
            double coef;                                  /* F_i = coef * d */
            if (r0 == 0.0)
                coef = 2.0 * k;
            else
                coef = r > 0.0 ? 2.0 * k * (r - r0) / r : 0.0;
            for (int a = 0; a < 3; ++a)
                F[3 * i + a] += coef * d[a];
            e += k * (r - r0) * (r - r0);
        }
    }
    if (E)
        *E = 0.5 * e;                                     /* each bond seen twice */
}

/* O8A: minimum-image vector x_j - x_i. */
static void min_image_vec(const double* R, int64_t i, int64_t j, const double L[3], double d[3])
{
    for (int a = 0; a < 3; ++a) {
        d[a] = R[3 * j + a] - R[3 * i + a];
        d[a] -= L[a] * nearbyint(d[a] / L[a]);
    }
}

/* O8A: energy and dU/dcos(theta) of one triplet from its two arm vectors. */
static void angle_terms(const double a[3], const double b[3], double k, double theta0, int32_t form,
                        double* U, double* dUdc, double* c_out, double* la, double* lb)
{
    const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double nb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const double dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
    const double cr = sqrt(cx * cx + cy * cy + cz * cz);
    const double c = dot / (na * nb);
    const double theta = atan2(cr, dot);
    if (form == 0) {
        double st = cr / (na * nb);
        if (st < 1e-3)
            st = 1e-3;
        *U = k * (theta - theta0) * (theta - theta0);
        *dUdc = -2.0 * k * (theta - theta0) / st;
    } else {
        const double c0 = cos(theta0);
        *U = k * (c - c0) * (c - c0);
        *dUdc = 2.0 * k * (c - c0);
    }
    *c_out = c;
    *la = na;
    *lb = nb;
}

void or_angles(const double* R, int64_t N, const int32_t* angles, int32_t A, int32_t ntypes,
               const double* k, const double* theta0, const int32_t* form, const double L[3], double* F,
               double* E)
{
    double e = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        for (int32_t r = 0; r < A; ++r) {
            const int32_t p = angles[(3 * (int64_t)r + 0) * N + i];
            const int32_t q = angles[(3 * (int64_t)r + 1) * N + i];
            const int32_t code = angles[(3 * (int64_t)r + 2) * N + i];
            const int32_t role = code & 1, type = code >> 1;
            if (p < 0 || type >= ntypes)
                continue;
            /* the triplet (end1, middle, end2) and which member this bead is */
            const int64_t mid = role == 1 ? i : p;
            const int64_t e1 = role == 1 ? p : i;
            const int64_t e2 = q;
            double a[3], b[3], U, dUdc, c, la, lb;
            min_image_vec(R, mid, e1, L, a);
            min_image_vec(R, mid, e2, L, b);
            angle_terms(a, b, k[type], theta0[type], form[type], &U, &dUdc, &c, &la, &lb);
            /* dc/dx_e1 = (b^ - c a^) / |a|, dc/dx_e2 = (a^ - c b^) / |b|, dc/dx_mid = -(sum) */
            double g1[3], g2[3];
            for (int d = 0; d < 3; ++d) {
                g1[d] = (b[d] / lb - c * a[d] / la) / la;
                g2[d] = (a[d] / la - c * b[d] / lb) / lb;
            }
            for (int d = 0; d < 3; ++d) {
                const double g = role == 1 ? -(g1[d] + g2[d]) : g1[d];
                F[3 * i + d] -= dUdc * g;
            }
            e += U;
        }
    }
    if (E)
        *E = e / 3.0;                                     /* each angle seen three times */
}

static double wrap_coord(double x, double L)
{
    double r = fmod(x, L);
    if (r < 0.0)
        r += L;
    if (r >= L)
        r = 0.0;
    return r;
}

void or_verlet_half1(double* R, double* V, const double* F, const double* inv_mass,
                     int64_t N, double dt, const double L[3])
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double im = inv_mass ? inv_mass[i] : 1.0;
        for (int a = 0; a < 3; ++a) {
            V[3 * i + a] += 0.5 * dt * F[3 * i + a] * im;
            R[3 * i + a] = wrap_coord(R[3 * i + a] + dt * V[3 * i + a], L[a]);
        }
    }
}

void or_verlet_half2(double* V, const double* F, const double* inv_mass, int64_t N,
                     double dt, double* out4)
{
    double ke = 0.0, px = 0.0, py = 0.0, pz = 0.0;
#pragma omp parallel for reduction(+ : ke, px, py, pz) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double im = inv_mass ? inv_mass[i] : 1.0;
        double mass = 1.0 / im;
        for (int a = 0; a < 3; ++a) {
            V[3 * i + a] += 0.5 * dt * F[3 * i + a] * im;
            ke += 0.5 * mass * V[3 * i + a] * V[3 * i + a];
        }
        px += mass * V[3 * i + 0];
        py += mass * V[3 * i + 1];
        pz += mass * V[3 * i + 2];
    }
    if (out4) {
        out4[0] = ke;
        out4[1] = px;
        out4[2] = py;
        out4[3] = pz;
    }
}

int64_t or_forces(const double* R, const uint8_t* T, int64_t N, const or_params_t* p,
                  double* F_field, double* F_bond, double* energies2)
{
    const or_mesh_t* m = p->mesh;
    const int64_t nm = (int64_t)m->M[0] * m->M[1] * m->M[2];
    uint64_t* counts = calloc((size_t)(p->K * nm), sizeof(uint64_t));
    double* V = malloc(sizeof(double) * (size_t)(p->K * nm));
    double* G = malloc(sizeof(double) * (size_t)(3 * p->K * nm));
    if (!counts || !V || !G) {
        free(counts);
        free(V);
        free(G);
        return -1;
    }
    double W = 0.0, Eb = 0.0;
    int64_t skipped = or_density(R, T, N, m, p->K, counts);
    or_potential(counts, m, N, p->K, p->kT, p->inv_kappa, p->chi, V, &W);
    or_gradient(V, m, p->K, G);
    or_gather(R, T, N, m, p->K, G, F_field);
    memset(F_bond, 0, sizeof(double) * (size_t)(3 * N));
    or_bonds(R, N, p->bonds, p->D, p->k_bond, p->r0, m->L, F_bond, &Eb);
    if (energies2) {
        energies2[0] = W;
        energies2[1] = Eb;
    }
    free(counts);
    free(V);
    free(G);
    return skipped;
}

static double kinetic(const double* V, const double* inv_mass, int64_t N)
{
    double ke = 0.0;
#pragma omp parallel for reduction(+ : ke) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double mass = inv_mass ? 1.0 / inv_mass[i] : 1.0;
        for (int a = 0; a < 3; ++a)
            ke += 0.5 * mass * V[3 * i + a] * V[3 * i + a];
    }
    return ke;
}

int or_run(double* R, double* V, const uint8_t* T, const double* inv_mass, int64_t N,
           const or_params_t* p, double dt, int32_t n_steps, double* energies)
{
    double* Ff = malloc(sizeof(double) * (size_t)(3 * N + 1));
    double* Fb = malloc(sizeof(double) * (size_t)(3 * N + 1));
    double* F = malloc(sizeof(double) * (size_t)(3 * N + 1));
    if (!Ff || !Fb || !F) {
        free(Ff);
        free(Fb);
        free(F);
        return -1;
    }
    double e2[2];
    int rc = 0;
    if (or_forces(R, T, N, p, Ff, Fb, e2) < 0)
        rc = -1;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < 3 * N; ++j)
        F[j] = Ff[j] + Fb[j];
    double ke = kinetic(V, inv_mass, N);
    energies[0] = ke;
    energies[1] = e2[1];
    energies[2] = e2[0];
    energies[3] = ke + e2[0] + e2[1];
    for (int32_t s = 1; s <= n_steps && rc == 0; ++s) {
        double out4[4];
        or_verlet_half1(R, V, F, inv_mass, N, dt, p->mesh->L);
        if (or_forces(R, T, N, p, Ff, Fb, e2) < 0)
            rc = -1;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < 3 * N; ++j)
            F[j] = Ff[j] + Fb[j];
        or_verlet_half2(V, F, inv_mass, N, dt, out4);
        double* e = energies + 4 * (int64_t)s;
        e[0] = out4[0];
        e[1] = e2[1];
        e[2] = e2[0];
        e[3] = out4[0] + e2[0] + e2[1];
    }
    free(Ff);
    free(Fb);
    free(F);
    return rc;
}

int or_run_interval(double* R, double* V, const uint8_t* T, const double* inv_mass, int64_t N,
                    const or_params_t* p, double dt, int32_t n_steps, int32_t field_every, double* energies)
{
    if (field_every < 1)
        return -2;
    const or_mesh_t* m = p->mesh;
    const int64_t nm = (int64_t)m->M[0] * m->M[1] * m->M[2];
    uint64_t* counts = malloc(sizeof(uint64_t) * (size_t)(p->K * nm));
    double* Vf = malloc(sizeof(double) * (size_t)(p->K * nm));
    double* G = malloc(sizeof(double) * (size_t)(3 * p->K * nm));
    double* Ff = malloc(sizeof(double) * (size_t)(3 * N + 1));
    double* Fb = malloc(sizeof(double) * (size_t)(3 * N + 1));
    double* F = malloc(sizeof(double) * (size_t)(3 * N + 1));
    int rc = (counts && Vf && G && Ff && Fb && F) ? 0 : -1;
    double W = 0.0;
    for (int32_t s = 0; s <= n_steps && rc == 0; ++s) {
        if (s > 0)
            or_verlet_half1(R, V, F, inv_mass, N, dt, m->L);
        if (s % field_every == 0) {
            /* rebuild the field from the current positions */
            memset(counts, 0, sizeof(uint64_t) * (size_t)(p->K * nm));
            or_density(R, T, N, m, p->K, counts);
            or_potential(counts, m, N, p->K, p->kT, p->inv_kappa, p->chi, Vf, &W);
            or_gradient(Vf, m, p->K, G);
        }
        or_gather(R, T, N, m, p->K, G, Ff);
        double Eb = 0.0;
        memset(Fb, 0, sizeof(double) * (size_t)(3 * N));
        or_bonds(R, N, p->bonds, p->D, p->k_bond, p->r0, m->L, Fb, &Eb);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < 3 * N; ++j)
            F[j] = Ff[j] + Fb[j];
        double ke;
        if (s > 0) {
            double out4[4];
            or_verlet_half2(V, F, inv_mass, N, dt, out4);
            ke = out4[0];
        } else {
            ke = kinetic(V, inv_mass, N);
        }
        double* e = energies + 4 * (int64_t)s;
        e[0] = ke;
        e[1] = Eb;
        e[2] = W;
        e[3] = ke + W + Eb;
    }
    free(counts);
    free(Vf);
    free(G);
    free(Ff);
    free(Fb);
    free(F);
    return rc;
}

/* O12: Philox4x32-10. Each round multiplies counter words 0 and 2 by the two
 * round constants into 64-bit products; the new counter is (high word of the
 * second product ^ word 1 ^ key 0, its low word, high word of the first
 * product ^ word 3 ^ key 1, its low word). Between rounds the key advances by
 * the two Weyl constants (golden ratio and sqrt(3) - 1, times 2^32). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint64_t MUL0 = 0xD2511F53u, MUL1 = 0xCD9E8D57u;
    const uint32_t WEYL0 = 0x9E3779B9u, WEYL1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += WEYL0;
            k1 += WEYL1;
        }
        const uint64_t p0 = MUL0 * (uint64_t)c[0];
        const uint64_t p1 = MUL1 * (uint64_t)c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        const uint32_t n3 = (uint32_t)p0;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
    }
    for (int j = 0; j < 4; ++j)
        out[j] = c[j];
}

static const double TWO_M24 = 1.0 / 16777216.0;     /* 2^-24 */

/* O13: one bead's draw at (tag, step): collision decision and, if it collides,
 * three standard normal deviates (Box-Muller, FP64). */
static int andersen_draw(int32_t tag, int64_t step, uint64_t seed, uint32_t thr, double g[3])
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)tag, (uint32_t)(uint64_t)step, (uint32_t)((uint64_t)step >> 32), 0u};
    uint32_t r[4], r2[4];
    or_philox4x32_10(ctr, key, r);
    if ((r[0] >> 8) >= thr)
        return 0;
    ctr[3] = 1u;
    or_philox4x32_10(ctr, key, r2);
    const double pi = 3.14159265358979323846;
    const double u1 = (double)((r[1] >> 8) + 1u) * TWO_M24;     /* (0, 1] */
    const double u2 = (double)(r[2] >> 8) * TWO_M24;            /* [0, 1) */
    const double u3 = (double)((r[3] >> 8) + 1u) * TWO_M24;
    const double u4 = (double)(r2[0] >> 8) * TWO_M24;
    const double rad1 = sqrt(-2.0 * log(u1));
    const double rad2 = sqrt(-2.0 * log(u3));
    g[0] = rad1 * cos(2.0 * pi * u2);
    g[1] = rad1 * sin(2.0 * pi * u2);
    g[2] = rad2 * cos(2.0 * pi * u4);
    return 1;
}

/* Integer threshold of a collision probability p in [0, 1]: floor(p 2^24). */
static uint32_t andersen_threshold(float p)
{
    if (!(p > 0.0f))
        return 0u;
    if (p >= 1.0f)
        return 1u << 24;
    return (uint32_t)floor((double)p * 16777216.0);
}

int64_t or_andersen(double* V, const int32_t* tag, const double* inv_mass, int64_t N, double kT,
                    float p, uint64_t seed, int64_t step, uint8_t* mask)
{
    const uint32_t thr = andersen_threshold(p);
    int64_t n = 0;
    for (int64_t i = 0; i < N; ++i) {
        double g[3];
        const int hit = andersen_draw(tag[i], step, seed, thr, g);
        if (mask)
            mask[i] = (uint8_t)hit;
        if (!hit)
            continue;
        const double sd = sqrt(kT * (inv_mass ? inv_mass[i] : 1.0));
        for (int a = 0; a < 3; ++a)
            V[3 * i + a] = sd * g[a];
        ++n;
    }
    return n;
}

int or_run_nvt(double* R, double* V, const uint8_t* T, const int32_t* tag, const double* inv_mass,
               int64_t N, const or_params_t* p, double dt, int32_t n_steps, int32_t field_every,
               double kT, float p_coll, uint64_t seed, double* energies)
{
    if (field_every < 1)
        return -2;
    const or_mesh_t* m = p->mesh;
    const int64_t nm = (int64_t)m->M[0] * m->M[1] * m->M[2];
    uint64_t* counts = malloc(sizeof(uint64_t) * (size_t)(p->K * nm));
    double* Vf = malloc(sizeof(double) * (size_t)(p->K * nm));
    double* G = malloc(sizeof(double) * (size_t)(3 * p->K * nm));
    double* Ff = malloc(sizeof(double) * (size_t)(3 * N + 1));
    double* Fb = malloc(sizeof(double) * (size_t)(3 * N + 1));
    double* F = malloc(sizeof(double) * (size_t)(3 * N + 1));
    int rc = (counts && Vf && G && Ff && Fb && F) ? 0 : -1;
    double W = 0.0;
    for (int32_t s = 0; s <= n_steps && rc == 0; ++s) {
        if (s > 0)
            or_verlet_half1(R, V, F, inv_mass, N, dt, m->L);
        if (s % field_every == 0) {
            memset(counts, 0, sizeof(uint64_t) * (size_t)(p->K * nm));
            or_density(R, T, N, m, p->K, counts);
            or_potential(counts, m, N, p->K, p->kT, p->inv_kappa, p->chi, Vf, &W);
            or_gradient(Vf, m, p->K, G);
        }
        or_gather(R, T, N, m, p->K, G, Ff);
        double Eb = 0.0;
        memset(Fb, 0, sizeof(double) * (size_t)(3 * N));
        or_bonds(R, N, p->bonds, p->D, p->k_bond, p->r0, m->L, Fb, &Eb);
        for (int64_t j = 0; j < 3 * N; ++j)
            F[j] = Ff[j] + Fb[j];
        if (s > 0) {
            or_verlet_half2(V, F, inv_mass, N, dt, NULL);
            or_andersen(V, tag, inv_mass, N, kT, p_coll, seed, s, NULL);
        }
        const double ke = kinetic(V, inv_mass, N);
        double* e = energies + 4 * (int64_t)s;
        e[0] = ke;
        e[1] = Eb;
        e[2] = W;
        e[3] = ke + W + Eb;
    }
    free(counts);
    free(Vf);
    free(G);
    free(Ff);
    free(Fb);
    free(F);
    return rc;
}

typedef struct {
    uint32_t key;
    int32_t tag;
    int64_t idx;
} sort_item;

static int cmp_item(const void* a, const void* b)
{
    const sort_item* x = a;
    const sort_item* y = b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    if (x->tag != y->tag)
        return x->tag < y->tag ? -1 : 1;
    return 0;
}

int or_sort_perm(const double* R, const int32_t* tag, int64_t N, const or_mesh_t* m,
                 int32_t B, int64_t* perm, uint32_t* keys)
{
    sort_item* it = malloc(sizeof(sort_item) * (size_t)(N > 0 ? N : 1));
    if (!it)
        return -1;
    int32_t nb[3];
    for (int d = 0; d < 3; ++d)
        nb[d] = (m->M[d] + B - 1) / B;
    for (int64_t i = 0; i < N; ++i) {
        int32_t c[3];
        uint32_t w[3][2];
        uint32_t key = 0xFFFFFFFFu;
        if (!bead_cell(R, i, m, c, w))
            key = ((uint32_t)(c[2] / B) * (uint32_t)nb[1] + (uint32_t)(c[1] / B)) * (uint32_t)nb[0] +
                  (uint32_t)(c[0] / B);
        it[i].key = key;
        it[i].tag = tag[i];
        it[i].idx = i;
        if (keys)
            keys[i] = key;
    }
    qsort(it, (size_t)N, sizeof(sort_item), cmp_item);
    for (int64_t i = 0; i < N; ++i)
        perm[i] = it[i].idx;
    free(it);
    return 0;
}
