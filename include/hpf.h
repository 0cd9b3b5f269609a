/*
 * hpf.h -- C ABI of libhpf, the MI355X (gfx950) hybrid particle-field MD step.
 *
 * The library computes one timestep of hybrid particle-field molecular
 * dynamics (hPF-MD; "MD-SCF" in Zhu et al., GALAMOST, arXiv 1310.2041):
 * beads deposit onto a periodic density mesh, a local field potential is
 * built from the Flory-Huggins chi matrix and a compressibility term, its
 * mesh gradient is interpolated back onto the beads as forces, harmonic bond
 * forces are added and velocity Verlet advances the system.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers to memory owned by the caller
 *    (hipMalloc or a framework allocator). The library never allocates and
 *    never frees them. Small parameter structs and the box array are HOST
 *    pointers, read during the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call only enqueues work on it and returns; results are valid once
 *    the stream has reached that point.
 *  - Bead arrays are structure-of-arrays, one row per bead, in storage order
 *    i = 0..N-1: positions R, velocities Vel and forces F are float[N][3]
 *    (x, y, z; 12 bytes per bead, no padding). Types T are uint8[N] in
 *    [0, K).
 *  - Mesh arrays are [K][Mz][My][Mx] with x fastest. A mesh point is a cell
 *    corner; the mesh is periodic, so there are as many points as cells.
 *  - Return value: HPF_OK, or a negative hpf_status_t for errors detected on
 *    the host before anything is enqueued (nothing is enqueued then).
 *    Conditions that only the device can see (a bead that cannot be binned,
 *    a mesh count near overflow, a non-finite coordinate after an update)
 *    set sticky bits that hpf_get_device_status() reads.
 *  - No C++ exception crosses this interface.
 *  - Results do not depend on the order in which beads are stored, except
 *    for the rounding order of FP64 energy sums; hpf_sort_by_cell() produces
 *    a canonical order, after which every result is bitwise reproducible.
 */
#ifndef HPF_H
#define HPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HPF_ABI_VERSION 1
#define HPF_FIX_BITS 16     /* S: fractional bits of a 1-D cloud-in-cell weight */
#define HPF_MAX_TYPES 8     /* K <= 8 species */
#define HPF_NPART 4096      /* slots per component of an FP64 partial-sum buffer */
#define HPF_MAX_BONDS 16    /* D <= 16 bond-table rows */
#define HPF_MAX_ANGLES 16   /* A <= 16 angle slots per bead */
#define HPF_MAX_ANGLE_TYPES 8

typedef int32_t hpf_status_t;
#define HPF_OK 0
#define HPF_EINVAL (-1)     /* an argument is invalid (null pointer, bad size or mesh) */
#define HPF_EHIP (-2)       /* the HIP runtime reported an error while enqueueing */
#define HPF_ESPACE (-3)     /* a caller-provided workspace is too small */
#define HPF_ETOOBIG (-4)    /* the problem needs more than HPF_STATIC_SCRATCH_BYTES */

/* Size of the fixed device scratch of hpf_density_scatter_cells_static. */
#define HPF_STATIC_SCRATCH_BYTES (32u << 20)

/* Sticky device status bits (hpf_get_device_status). */
#define HPF_FLAG_BAD_BEAD 0x1u   /* a bead with a non-finite or out-of-range position
                                    (|x*s| >= 2^24) or a type >= K was skipped */
#define HPF_FLAG_OVERFLOW 0x2u   /* a mesh count reached 2^62 (risk of u64 wrap) */
#define HPF_FLAG_NONFINITE 0x4u  /* verlet_step produced a non-finite coordinate */
#define HPF_FLAG_BAD_BOND 0x8u   /* a bond-table entry was outside [-1, N) */
#define HPF_FLAG_SORT_ORDER 0x10u /* hpf_sort_by_cell got tags that are not a permutation
                                     of [0, N); its output is not a valid permutation */

/* Periodic box and density mesh.
 *  L      box edge lengths, > 0.
 *  M      mesh points (= cells) per edge, >= 3.
 *  s      cells per unit length, fl32(M / L): the bead coordinate in cell
 *         units is u = fl32(x * s) (one IEEE single rounding).
 *  c_norm volume fraction per fixed-point count, 1 / (2^48 rho0 dV) with
 *         rho0 = N / (Lx Ly Lz) and dV = Lx Ly Lz / (Mx My Mz); i.e.
 *         Mx My Mz / (2^48 N). 0 when N = 0.
 * hpf_mesh_make() fills s and c_norm from L, M and N. */
typedef struct hpf_mesh {
    float L[3];
    int32_t M[3];
    float s[3];
    int32_t reserved;
    double c_norm;
} hpf_mesh_t;

/* Field parameters of eq. (4) (MD-SCF section):
 *   V_K = kT sum_K' chi[K][K'] phi_K' + inv_kappa (sum_K phi_K - 1).
 * chi is row-major K x K (entry [a*K + b]); it should be symmetric. */
typedef struct hpf_field {
    int32_t K;
    int32_t reserved;
    double kT;
    double inv_kappa;
    double chi[HPF_MAX_TYPES * HPF_MAX_TYPES];
} hpf_field_t;

/* Andersen thermostat (Integration methods section: NVT with the Andersen
 * thermostat). At time level n each bead collides with the heat bath with
 * probability p and then takes a new velocity from the Maxwell distribution at
 * kT: v = sqrt(kT / m) (g0, g1, g2). The decision and the deviates come from the
 * counter-based generator Philox4x32-10 (Salmon et al., SC'11) with key `seed`
 * and counters (tag_i + tag_offset, n, 0) and (tag_i + tag_offset, n, 1): the bead collides when
 * (r0 >> 8) < floor(p 2^24); g0, g1 are the Box-Muller pair of the 24-bit
 * uniforms of r1 and r2 (((r1 >> 8) + 1) 2^-24 under the logarithm), g2 the
 * cosine deviate of r3 and of word 0 of the second counter. Draws therefore
 * depend only on (seed, tag, n), not on the storage order or launch shape.
 *  p     collision probability per step (collision rate x dt), in [0, 1];
 *        0 = no thermostat.
 *  kT    bath temperature, > 0.
 *  step  DEVICE pointer to the time level n (int64), read by the kernels when
 *        they run, so that a captured graph sees the value the caller has
 *        advanced in the meantime (the library never writes it).
 *  tag   DEVICE int32[N], the beads' tags in their current storage order.
 *  tag_offset  added (mod 2^32) to every tag to form the generator's first
 *        counter word. A batch of replicas numbers its tags globally, replica r
 *        from its first bead on; a system run alone with tags 0..N_r-1 and
 *        tag_offset = that first bead draws the same numbers as replica r.
 * A null thermostat pointer is no thermostat. Invalid values give HPF_EINVAL. */
typedef struct hpf_thermostat {
    float p;
    float kT;
    uint64_t seed;
    const int64_t* step;
    const int32_t* tag;
    int64_t tag_offset;
} hpf_thermostat_t;

/* Library ABI version (HPF_ABI_VERSION). */
int32_t hpf_abi_version(void);

/* Human-readable text for a status code. */
const char* hpf_status_string(hpf_status_t status);

/* Host helper: fill `out` from box edges L[3] (host), mesh sizes M[3] (host)
 * and the bead count N >= 0. Returns HPF_EINVAL for L <= 0 or M < 3. */
hpf_status_t hpf_mesh_make(const float* L, const int32_t* M, int64_t n_beads,
                           hpf_mesh_t* out);

/* ---------------------------------------------------------------------------
 * hpf_density_scatter -- density assignment (MD-SCF section: every bead
 * spreads its density fractions over the eight vertices of its cell;
 * Algorithm 1 Kernels 1-2 compute the same sums by gathering).
 *
 * For bead i with u_d = fl32(x_d * s_d), c_d = floor(u_d) mod M_d,
 * f_d = fl32(u_d - floor(u_d)), q_d = floor(f_d * 2^16), the 1-D weights are
 * (2^16 - q_d, q_d) and vertex c + a (a in {0,1}^3, periodic) receives the
 * product W_a of its three 1-D weights; the eight W_a sum to 2^48.
 *   counts[T_i][c + a] += W_a        (uint64, exact, order independent)
 *
 * R       float[N][3] device; T uint8[N] device; N >= 0.
 * mesh    host; K in [1, HPF_MAX_TYPES].
 * counts  uint64[K][Mz][My][Mx] device, ACCUMULATED into (zero it first, or
 *         let hpf_field_potential clear it after reading).
 * Beads with a non-finite position, |u_d| >= 2^24 or T_i >= K are skipped
 * and set HPF_FLAG_BAD_BEAD. Fastest when beads are stored in cell order
 * (hpf_sort_by_cell); correct for any order.
 * ------------------------------------------------------------------------- */
hpf_status_t hpf_density_scatter(const float* R, const uint8_t* T, int64_t N,
                                 const hpf_mesh_t* mesh, int32_t K, uint64_t* counts,
                                 void* stream);

/* ---------------------------------------------------------------------------
 * hpf_density_scatter_cells -- the same counts as hpf_density_scatter, for
 * beads stored in the order of hpf_sort_by_cell (positions may have moved
 * since that sort). The paper computes these sums by gathering at the mesh
 * points over a cell list (Algorithm 1 Kernel 2); here each B^3 brick of cells
 * deposits its listed beads into an LDS box of (B + 1 + 2*halo)^3 points that
 * is stored to a per-brick partial buffer, and one thread per mesh point adds
 * the boxes covering it. Beads that moved more than `halo` cells out of their
 * brick since the sort, and beads the sort could not bin, are added
 * afterwards with global atomics. Counts are exact for any drift.
 *
 * cell_start  uint32[NK + 2] device, from the hpf_sort_by_cell call that
 *             produced the current storage order, with the same B.
 * B           brick edge 3..16 (0 selects 8); halo 0..2 cells, halo < B. Every
 *             M_d must be >= B + 1 + 2*halo, and K (B + 1 + 2 halo)^3 * 8 bytes
 *             must fit in 160 KiB of LDS (HPF_EINVAL otherwise).
 * counts      uint64[K][Mz][My][Mx] device, OVERWRITTEN (need not be zero).
 * work        device workspace of at least
 *             hpf_scatter_workspace_bytes(N, mesh, K, B, halo) bytes (stray
 *             list and partial boxes); 0 from that call means invalid sizes.
 * Skipped beads set HPF_FLAG_BAD_BEAD as in hpf_density_scatter.
 * ------------------------------------------------------------------------- */
size_t hpf_scatter_workspace_bytes(int64_t N, const hpf_mesh_t* mesh, int32_t K, int32_t B,
                                   int32_t halo);
hpf_status_t hpf_density_scatter_cells(const float* R, const uint8_t* T, int64_t N,
                                       const hpf_mesh_t* mesh, int32_t K,
                                       const uint32_t* cell_start, int32_t B, int32_t halo,
                                       uint64_t* counts, void* work, size_t work_bytes,
                                       void* stream);

/* ---------------------------------------------------------------------------
 * hpf_density_scatter_cells_static -- hpf_density_scatter_cells for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same counts, from the same
 * kernels, with no workspace argument. The stray list and partial boxes live in
 * a fixed device array of HPF_STATIC_SCRATCH_BYTES (32 MiB) that each GPU holds
 * while the library is loaded; the call allocates nothing.
 *
 * Arguments are those of hpf_density_scatter_cells without work/work_bytes.
 * Returns HPF_ETOOBIG, with nothing enqueued, when
 * hpf_scatter_workspace_bytes(N, mesh, K, B, halo) exceeds
 * HPF_STATIC_SCRATCH_BYTES (for example 1M beads on a 64^3 mesh with K = 2,
 * B = 8, halo = 2 needs 22 MB; 10M beads on 128^3 need 184 MB and are refused).
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * behind (each launch clears what must start at zero): calls that overlap in
 * time on one GPU, from any streams or threads, race and must not be made.
 * ------------------------------------------------------------------------- */
hpf_status_t hpf_density_scatter_cells_static(const float* R, const uint8_t* T, int64_t N,
                                              const hpf_mesh_t* mesh, int32_t K,
                                              const uint32_t* cell_start, int32_t B, int32_t halo,
                                              uint64_t* counts, void* stream);

/* ---------------------------------------------------------------------------
 * hpf_field_potential -- external potential of eq. (4) at every mesh point.
 *
 *   phi_K = counts_K * c_norm                  (FP64)
 *   V_K   = kT sum_K' chi[K][K'] phi_K' + inv_kappa (sum_K phi_K - 1)
 * computed in FP64 and stored as FP32; counts are then set to 0 (read and
 * clear), so the next scatter can accumulate into them.
 *
 * counts  uint64[K][M^3] device, read then zeroed.
 * V       float[K][M^3] device, overwritten.
 * w_part  nullable, double[HPF_NPART] device: receives partial sums of the
 *         field energy W = rho0 dV sum_v [ kT/2 sum_KK' chi phi_K phi_K'
 *         + inv_kappa/2 (sum_K phi_K - 1)^2 ] (the functional whose
 *         derivative by the bead count at v is V_K(v)); reduce with
 *         hpf_reduce_partials(w_part, 1, ...).
 * present nullable uint8[M^3] device: the composition list of every mesh point
 *         (the MD-SCF section's list of the components present, here per point):
 *         bit K is set when counts_K > 0 there. hpf_field_gradient uses it to
 *         skip the species that are absent (dilute multi-component systems).
 * A count >= 2^62 sets HPF_FLAG_OVERFLOW.
 * ------------------------------------------------------------------------- */
hpf_status_t hpf_field_potential(uint64_t* counts, const hpf_mesh_t* mesh,
                                 const hpf_field_t* field, float* V, double* w_part,
                                 uint8_t* present, void* stream);

/* ---------------------------------------------------------------------------
 * hpf_field_gradient -- mesh gradient of the potential (Algorithm 1
 * Kernel 3, read as a centred periodic difference at the mesh point):
 *   G_K(v) = ( (V_K(v+e_x) - V_K(v-e_x)) / (2 h_x), ... y, ... z )
 * with 1/(2 h_d) = s_d / 2.
 *
 * V  float[K][M^3] device.  G float[K][M^3][3] device, overwritten.
 * present  nullable uint8[M^3] device, the composition list that
 *          hpf_field_potential wrote for the same counts: G_K(v) is then written
 *          only where bit K of present[v] is set; the other entries keep their
 *          previous values (they must be finite, e.g. zero at first). The force
 *          gathers read G_K only at mesh points where a bead of species K has a
 *          non-zero weight, all of which carry bit K, so forces are unchanged.
 * ------------------------------------------------------------------------- */
hpf_status_t hpf_field_gradient(const float* V, const hpf_mesh_t* mesh, int32_t K,
                                float* G, const uint8_t* present, void* stream);

/* ---------------------------------------------------------------------------
 * hpf_force_gather -- field force on every bead, eq. (6) (Algorithm 1
 * Kernel 4, read as interpolation with the density-assignment weights):
 *   F_i = - sum_a (W_a(i) / 2^48) G_{T_i}(c_i + a)
 *
 * R float[N][3], T uint8[N], G float[K][M^3][3] device.
 * F float[N][3] device, OVERWRITTEN. Skipped beads (see
 * hpf_density_scatter) get F = 0.
 * ------------------------------------------------------------------------- */
hpf_status_t hpf_force_gather(const float* R, const uint8_t* T, int64_t N,
                              const hpf_mesh_t* mesh, int32_t K, const float* G, float* F,
                              void* stream);

/* ---------------------------------------------------------------------------
 * hpf_force_gather_staggered -- the field force of eq. (6) read literally from
 * Algorithm 1: Kernel 3's staggered backward and forward differences, taken at
 * the bead's nearest mesh point and blended with Kernel 4's fraction ratios.
 * Per axis d, with u_d, c_d and q_d as in hpf_density_scatter: the nearest point
 * is n_d = c_d when q_d < 2^15, else c_d + 1 (periodic), delta_d = (q_d or
 * q_d - 2^16) / 2^16 in [-1/2, 1/2), and
 *   F_i,d = -s_d [ (1/2 - delta_d)(V_T(n) - V_T(n - e_d))
 *                + (1/2 + delta_d)(V_T(n + e_d) - V_T(n)) ],   T = T_i,
 * the sum over species of Kernel 4 being contained in V (the equation is
 * linear). No transverse interpolation; unlike hpf_force_gather this is not
 * the transpose of the density assignment, so it does not conserve momentum
 * exactly. It needs no gradient mesh.
 *
 * R float[N][3], T uint8[N], V float[K][M^3] device (hpf_field_potential).
 * F float[N][3] device, OVERWRITTEN. Skipped beads (see
 * hpf_density_scatter) get F = 0.
 * ------------------------------------------------------------------------- */
hpf_status_t hpf_force_gather_staggered(const float* R, const uint8_t* T, int64_t N,
                                        const hpf_mesh_t* mesh, int32_t K, const float* V,
                                        float* F, void* stream);

/* ---------------------------------------------------------------------------
 * bond_forces -- harmonic bonds U = k (r - r0)^2 (eq. (7), no factor 1/2),
 * one thread per bead summing over its own bonds, so each bond is evaluated
 * from both ends (Bonded forces section). With d = minimum image of
 * x_j - x_i and r = |d|:  F_i += 2 k (r - r0) d / r  (r0 = 0: F_i += 2 k d;
 * r = 0 with r0 != 0: no force).
 *
 * bonds  int32[D][N] device, the table form of the paper: bonds[b*N + i] is
 *        the storage index of the b-th partner of bead i, -1 for none;
 *        D in [0, HPF_MAX_BONDS]. Entries outside [-1, N) are skipped and set
 *        HPF_FLAG_BAD_BOND.
 * box    host float[3], the periodic box edges.
 * F      float[N][3] device, ACCUMULATED into.
 * e_part nullable double[HPF_NPART] device: partial sums of the bond energy
 *        sum over bonds of k (r - r0)^2.
 * ------------------------------------------------------------------------- */
hpf_status_t bond_forces(const float* R, int64_t N, const int32_t* bonds, int32_t D,
                         float k, float r0, const float* box, float* F, double* e_part,
                         void* stream);

/* ---------------------------------------------------------------------------
 * angle_forces -- the angle potentials of the Bonded forces section,
 *   form 0:  U = k (theta - theta0)^2        form 1:  U = k (cos theta - cos theta0)^2
 * with theta the angle at the middle bead j of a triplet (i, j, k) between the
 * minimum-image vectors x_i - x_j and x_k - x_j. Stored like the bonds, per bead
 * (the paper keeps angles in the bond-table form, marking whether the bead is
 * the middle or an end, and evaluates each angle three times, once per member):
 *   angles[(3a + 0) N + i], angles[(3a + 1) N + i]  the other two members of bead
 *       i's a-th angle (-1 in the first = no angle);
 *   angles[(3a + 2) N + i] = role + 2 type: role 1 if bead i is the middle (the
 *       partners are the ends), 0 if it is an end (the first partner is then the
 *       middle, the second the other end); type < ntypes selects the parameters.
 * A in [0, HPF_MAX_ANGLES]; ntypes in [1, HPF_MAX_ANGLE_TYPES]; k, theta0 (radians)
 * and form (0 or 1) are HOST arrays of ntypes entries. For the harmonic form
 * dU/dcos = -2k (theta - theta0) / sin(theta), sin(theta) floored at 1e-3 (the
 * direction of the force of an exactly straight triplet is undefined).
 * F float[N][3] device, ACCUMULATED into. e_part nullable double[HPF_NPART]:
 * partial sums of the angle energy, each angle once. Entries outside [-1, N) or
 * with a type >= ntypes are skipped and set HPF_FLAG_BAD_BOND.
 * ------------------------------------------------------------------------- */
hpf_status_t angle_forces(const float* R, int64_t N, const int32_t* angles, int32_t A, int32_t ntypes,
                          const float* k, const float* theta0, const int32_t* form, const float* box,
                          float* F, double* e_part, void* stream);

/* ---------------------------------------------------------------------------
 * verlet_step -- velocity Verlet (Integration methods section), split into
 * its two half steps around the force evaluation:
 *   half = 1:  v += dt/2 F/m;  x += dt v;  x wrapped into [0, L)
 *   half = 2:  v += dt/2 F/m
 * inv_mass   nullable float[N] device (NULL = unit masses).
 * box        host float[3].  dt > 0.
 * kin_part   nullable double[4][HPF_NPART] device (half = 2 only): partial
 *            sums of {KE = sum m v^2 / 2, Px, Py, Pz} after the update.
 * A non-finite updated coordinate sets HPF_FLAG_NONFINITE.
 * ------------------------------------------------------------------------- */
hpf_status_t verlet_step(float* R, float* Vel, const float* F, const float* inv_mass,
                         int64_t N, float dt, const float* box, int32_t half,
                         double* kin_part, void* stream);

/* hpf_andersen -- the Andersen collisions of time level *thermostat->step on
 * every bead (see hpf_thermostat_t), to be applied after verlet_step(half = 2).
 * Vel float[N][3] device, updated; inv_mass nullable float[N] (NULL = unit
 * masses). kin_part nullable double[4][HPF_NPART]: partial sums of {KE, Px,
 * Py, Pz} after the collisions (as verlet_step's). thermostat must not be NULL. */
hpf_status_t hpf_andersen(float* Vel, const float* inv_mass, int64_t N,
                          const hpf_thermostat_t* thermostat, double* kin_part, void* stream);

/* ---------------------------------------------------------------------------
 * hpf_advance -- one fused pass over the beads that produces exactly the
 * results of this call sequence (bit for bit):
 *     hpf_force_gather(R, ..., F); bond_forces(R, ..., F, e_part);
 *     verlet_step(half = 2, kin_part); verlet_step(half = 1)
 * i.e. the field force (eq. 6) and bond forces (eq. 7) at x_n, the second
 * half kick of step n (kinetic-energy and momentum partials at v_n) and the
 * first half kick and drift of step n + 1 (Integration methods section).
 *
 * R       float[N][3] device, x_n, read only (bond partners are read here).
 * R_next  float[N][3] device, receives x_{n+1} wrapped into the box; must not
 *         alias R.
 * Vel     float[N][3] device, v_{n-1/2} in, v_{n+1/2} out.
 * G       float[K][M^3][3] device, the gradient mesh of x_n.
 * bonds, D, k, r0, box, inv_mass, dt: as in bond_forces / verlet_step.
 * F_out   nullable float[N][3] device: receives the total force at x_n.
 * e_part  nullable double[HPF_NPART]; kin_part nullable double[4][HPF_NPART]:
 *         as in bond_forces and verlet_step(half = 2).
 * thermostat  nullable: with it, the Andersen collisions of time level
 *         *thermostat->step act on v_n right after the second half kick, as
 *         hpf_andersen after verlet_step(half = 2) would, and the kinetic-energy
 *         partials are those of the velocities after the collisions.
 * Sets HPF_FLAG_BAD_BEAD / HPF_FLAG_BAD_BOND / HPF_FLAG_NONFINITE like the
 * separate calls.
 * ------------------------------------------------------------------------- */
hpf_status_t hpf_advance(const float* R, float* R_next, float* Vel, const uint8_t* T, int64_t N,
                         const hpf_mesh_t* mesh, int32_t K, const float* G, const int32_t* bonds,
                         int32_t D, float k, float r0, const float* box, const float* inv_mass,
                         float dt, float* F_out, double* e_part, double* kin_part,
                         const hpf_thermostat_t* thermostat, void* stream);

/* ---------------------------------------------------------------------------
 * hpf_advance_scatter -- hpf_advance (bit for bit the same bead updates) that
 * also deposits the new positions x_{n+1} for the next step's density (the
 * assignment of the MD-SCF section, Algorithm 1 Kernel 2), so the next step
 * need not read the beads again for it. One workgroup takes the beads one
 * brick listed at the last sort, advances them and adds the fixed-point
 * weights of their new positions to the brick's LDS deposit box, which is
 * stored to the brick's partial buffer in `work` (the layout that
 * hpf_density_scatter_cells uses). New positions more than `halo` cells out
 * of their brick, and beads the sort could not bin, are added to `counts`
 * with global atomics. hpf_density_finish_cells then adds the partial boxes
 * to `counts`; the result equals hpf_density_scatter(R_next) bit for bit.
 *
 * Arguments as in hpf_advance (thermostat included), plus:
 * cell_start, B, halo  as in hpf_density_scatter_cells (same limits).
 * counts  uint64[K][M^3] device, ADDED to; it must hold zeros (or counts to be
 *         kept) on entry. hpf_field_potential leaves it zeroed.
 * work    device workspace of at least hpf_scatter_workspace_bytes(N, mesh,
 *         K, B, halo) bytes (HPF_ESPACE otherwise); its partial boxes are
 *         overwritten and must not be touched before hpf_density_finish_cells.
 * The energy partials are grouped by workgroup, so their sums may differ from
 * hpf_advance's in the last FP64 bits; every bead state is identical.
 * Positions that cannot be binned set HPF_FLAG_BAD_BEAD.
 * ------------------------------------------------------------------------- */
hpf_status_t hpf_advance_scatter(const float* R, float* R_next, float* Vel, const uint8_t* T,
                                 int64_t N, const hpf_mesh_t* mesh, int32_t K, const float* G,
                                 const int32_t* bonds, int32_t D, float k, float r0,
                                 const float* box, const float* inv_mass, float dt,
                                 const uint32_t* cell_start, int32_t B, int32_t halo,
                                 uint64_t* counts, void* work, size_t work_bytes, float* F_out,
                                 double* e_part, double* kin_part,
                                 const hpf_thermostat_t* thermostat, void* stream);

/* hpf_density_finish_cells -- counts += the sum of the partial deposit boxes
 * that hpf_advance_scatter left in `work` (same N, mesh, K, B, halo), i.e.
 * the second pass of hpf_density_scatter_cells in accumulate form. After it,
 * `counts` holds the exact density counts of the positions that
 * hpf_advance_scatter produced, whatever the bead order in between (a
 * hpf_sort_by_cell call between the two does not change them). */
hpf_status_t hpf_density_finish_cells(uint64_t* counts, int64_t N, const hpf_mesh_t* mesh,
                                      int32_t K, int32_t B, int32_t halo, const void* work,
                                      size_t work_bytes, void* stream);

/* hpf_field_potential_cells -- hpf_density_finish_cells followed by
 * hpf_field_potential in one pass over the mesh (eq. (4) with the counts of
 * the positions hpf_advance_scatter deposited): each point's partial boxes
 * are added to the counts it holds, the counts are cleared and V written.
 * V is bitwise that of the two calls; w_part (nullable, double[HPF_NPART])
 * receives the field-energy partials, grouped per workgroup, so their sum may
 * differ from hpf_field_potential's in the last bits. N, mesh, B, halo and
 * work as in hpf_advance_scatter; K = field->K; present (nullable) as in
 * hpf_field_potential. */
hpf_status_t hpf_field_potential_cells(uint64_t* counts, int64_t N, const hpf_mesh_t* mesh,
                                       const hpf_field_t* field, int32_t B, int32_t halo,
                                       const void* work, size_t work_bytes, float* V,
                                       double* w_part, uint8_t* present, void* stream);

/* Deterministic FP64 reduction of partial-sum buffers: out[c] = sum of
 * part[c*HPF_NPART .. (c+1)*HPF_NPART) in a fixed tree order, c < ncomp.
 * part and out are device pointers; ncomp in [1, 8]. */
hpf_status_t hpf_reduce_partials(const double* part, int32_t ncomp, double* out,
                                 void* stream);

/* ---------------------------------------------------------------------------
 * hpf_sort_by_cell -- put beads in canonical cell-list order (the paper
 * reorders particle data for cache hits and bins beads into a cell list;
 * Algorithm 1 Kernel 1). The key of a bead is the brick of B^3 cells that
 * holds its cell, bricks numbered x fastest:
 *   key = (bz*NBy + by)*NBx + bx,  b_d = c_d / B,  NB_d = ceil(M_d / B).
 * Beads that cannot be binned get key NK = NBx*NBy*NBz and go last.
 * Output order: ascending (key, tag), so every brick's beads are one
 * contiguous range and, inside it, the beads of a chain (consecutive tags)
 * are neighbours. Positions, velocities, types and tags are permuted into the
 * *_out arrays and the bond table is permuted and its entries renumbered to
 * the new storage indices. The order comes from a stable counting sort of
 * the beads taken in tag order, so it does not depend on the input order.
 *
 * B            brick edge in cells, 1..16 (0 selects 8); NK + 1 must not
 *              exceed 36864 keys (HPF_EINVAL otherwise).
 * *_in / *_out device arrays of N rows (Vel/tag/bonds may be NULL together
 *              with their outputs; D may be 0); in and out must not alias.
 * tag_in       a permutation of [0, N) (the beads' original indices); NULL
 *              uses the input index. A tag outside [0, N) or a repeated tag
 *              sets HPF_FLAG_SORT_ORDER; the output is then not a valid
 *              permutation (every index written stays inside [0, N)).
 * cell_start   nullable uint32[NK + 2] device: cell_start[k] = index of the
 *              first bead with key >= k, i.e. brick k's beads are
 *              [cell_start[k], cell_start[k+1]); cell_start[NK] = number of
 *              binned beads, cell_start[NK+1] = N.
 * work         device workspace of at least hpf_sort_workspace_bytes()
 *              bytes (HPF_ESPACE otherwise).
 * ------------------------------------------------------------------------- */
size_t hpf_sort_workspace_bytes(int64_t N, const hpf_mesh_t* mesh, int32_t B);
hpf_status_t hpf_sort_by_cell(const hpf_mesh_t* mesh, int32_t B, int64_t N,
                              const float* R_in, const float* Vel_in, const uint8_t* T_in,
                              const int32_t* tag_in, const int32_t* bonds_in, int32_t D,
                              float* R_out, float* Vel_out, uint8_t* T_out, int32_t* tag_out,
                              int32_t* bonds_out, uint32_t* cell_start, void* work,
                              size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * hpf_resort_by_cell -- the order and outputs of hpf_sort_by_cell, for beads
 * that are in the order an earlier hpf_sort_by_cell / hpf_resort_by_cell with
 * the same mesh and B produced (positions may have moved since; the storage
 * order must not have changed). That sort's key starts come in as
 * cell_start_in. Between sorts most beads keep their brick, so the order is
 * built per brick rather than over the whole tag sequence: the beads that keep
 * their brick stay in tag order, the others are sorted by tag per new brick,
 * and the two lists are merged by tag. The work is a few passes in storage
 * order whatever the number of bricks.
 *
 * Arguments as hpf_sort_by_cell, plus:
 * cell_start_in   uint32[NK + 2] device, the earlier sort's key starts.
 * cell_start_out  uint32[NK + 2] device, the new key starts (must not alias
 *                 cell_start_in).
 * work            as for hpf_sort_by_cell (hpf_sort_workspace_bytes).
 * If the input is not in an earlier sort's order (a key range out of tag
 * order), HPF_FLAG_SORT_ORDER is set and the output, while a set of valid
 * indices, is not the sorted order.
 * ------------------------------------------------------------------------- */
hpf_status_t hpf_resort_by_cell(const hpf_mesh_t* mesh, int32_t B, int64_t N, const float* R_in,
                                const float* Vel_in, const uint8_t* T_in, const int32_t* tag_in,
                                const int32_t* bonds_in, int32_t D, float* R_out, float* Vel_out,
                                uint8_t* T_out, int32_t* tag_out, int32_t* bonds_out,
                                const uint32_t* cell_start_in, uint32_t* cell_start_out, void* work,
                                size_t work_bytes, void* stream);

/* hpf_sort_angles -- the per-bead angle table (angle_forces layout, int32[3A][N])
 * in the order of the hpf_sort_by_cell or hpf_resort_by_cell call that last used
 * `work` (same mesh, B and N, and `work` untouched since): rows are permuted with
 * their beads, the partner rows renumbered to the new storage indices, the code
 * rows kept. angles_out must not alias angles_in. Partners outside [-1, N) become
 * -1 and set HPF_FLAG_BAD_BOND. */
hpf_status_t hpf_sort_angles(const hpf_mesh_t* mesh, int32_t B, int64_t N, const int32_t* angles_in,
                             int32_t A, int32_t* angles_out, const void* work, size_t work_bytes,
                             void* stream);

/* ===========================================================================
 * Batched replicas (a phase-diagram sweep): many independent systems of
 * uneven size, box and chi advanced by one set of kernel launches per phase.
 *
 * The caller concatenates the replicas' beads (replica r owns storage indices
 * [bead_offset, bead_offset + n_beads), offsets contiguous and increasing; the
 * bond table is [D][N_total] with GLOBAL indices; tags must be unique and
 * increasing in the initial order) and provides two sets of bead buffers
 * (current / ping-pong), one concatenated mesh set (replica r's
 * [K][M_r^3] block follows replica r-1's, in replica order) and a workspace.
 * The batch sorts all replicas with one counting sort over disjoint key
 * ranges and runs the cell scatter, potential, gradient and fused advance as
 * one launch each over a work list of (replica, range) items. Each replica's
 * beads follow bit for bit the trajectory of the single-system calls; FP64
 * energy sums differ only in summation grouping.
 * ========================================================================= */
typedef struct hpf_replica {
    int64_t bead_offset;
    int64_t n_beads;
    float L[3];
    int32_t M[3];            /* each M_d >= brick + 5 */
    double kT;
    double inv_kappa;
    double chi[HPF_MAX_TYPES * HPF_MAX_TYPES];   /* row-major K x K */
} hpf_replica_t;

typedef struct hpf_batch_config {
    int32_t K;               /* species, same for all replicas */
    int32_t D;               /* bond-table rows */
    float k_bond, r0, dt;    /* eq. (7) and the time step, same for all replicas */
    int32_t brick;           /* sort brick edge B, 3..8 (0 selects 8) */
    int32_t halo;            /* cell-scatter drift halo, 0..2, < B */
    int32_t sort_every;      /* re-sort every n steps (0: never after start) */
    int32_t bead_chunk;      /* beads per work item, >= 512 */
    int32_t mesh_chunk;      /* mesh points per potential work item, >= 2048 */
    int32_t fuse_deposit;    /* 1: each step's fused pass also deposits the new positions
                                (as hpf_advance_scatter), so the next step only finishes
                                the density; 0: a separate cell scatter every step */
    float thermo_p;          /* Andersen collision probability per step (hpf_thermostat_t),
                                0 = NVE; each replica's bath is at its own kT */
    int32_t reserved;
    uint64_t thermo_seed;    /* generator key of the thermostat; the batch keeps the time
                                level on the device (1 at the first step after
                                hpf_batch_start) and advances it every step */
} hpf_batch_config_t;

typedef struct hpf_batch_buffers {
    float* R[2];             /* float[N_total][3] each */
    float* Vel[2];
    uint8_t* T[2];
    int32_t* tag[2];
    int32_t* bonds[2];       /* int32[D][N_total] each (NULL when D = 0) */
    uint64_t* counts;        /* sum_r K M_r^3 */
    float* V;                /* sum_r K M_r^3 */
    float* G;                /* sum_r K M_r^3 * 3 */
} hpf_batch_buffers_t;

typedef struct hpf_batch hpf_batch_t;   /* host object; owns no device memory */

/* Workspace bytes for these replicas and configuration (0 = invalid). */
size_t hpf_batch_workspace_bytes(const hpf_replica_t* reps, int32_t n_rep,
                                 const hpf_batch_config_t* cfg);
/* Build the replica table and work lists (synchronous host->device copies into
 * `work`). Buffers and workspace must outlive the batch and not move. The bond
 * table bufs->bonds[0] is read back once (synchronously): a partner outside its
 * own replica's bead range returns HPF_EINVAL. */
hpf_status_t hpf_batch_create(const hpf_replica_t* reps, int32_t n_rep,
                              const hpf_batch_config_t* cfg, const hpf_batch_buffers_t* bufs,
                              void* work, size_t work_bytes, hpf_batch_t** out);
/* Sort, forces at x_0 with energies, then the first half step. */
hpf_status_t hpf_batch_start(hpf_batch_t* batch, void* stream);
/* n_steps fused steps (sorting on the configured cadence); with report_last,
 * the energies of the last step are reduced per replica. */
hpf_status_t hpf_batch_step(hpf_batch_t* batch, int32_t n_steps, int32_t report_last,
                            void* stream);
/* Device pointers of the current bead buffers and of the per-replica energies
 * double[n_rep][8] = {KE, E_bond, W, E_tot, Px, Py, Pz, 0}. Any may be NULL. */
hpf_status_t hpf_batch_current(const hpf_batch_t* batch, float** R, float** Vel, uint8_t** T,
                               int32_t** tag, int32_t** bonds, double** energies);
/* Density counts of every replica at the current positions (the assignment of
 * the MD-SCF section, as hpf_density_scatter computes it per system), e.g. for
 * order parameters of a phase-diagram sweep. counts_out is uint64[K][sum_r M_r^3]
 * device (replica r's block at K * (sum of the earlier replicas' M^3)), OVERWRITTEN;
 * it must not be the batch's own counts buffer (HPF_EINVAL). The batch's state is
 * not changed, so stepping continues as if the call had not been made. */
hpf_status_t hpf_batch_density(hpf_batch_t* batch, uint64_t* counts_out, void* stream);
/* Autotuner of the launch shape on the live system. Candidates: the fused deposit
 * with deposit halo {1, 2} x sort interval {5, 10, 20, 30, 40}, and the separate
 * scatter with halo {1, 2} x bead_chunk {2048, 4096} (sort every 10). Each
 * candidate runs three times from a fresh sort for trial_steps steps (at least
 * 20) rounded up to a multiple of its sort interval; its time is the median of
 * the three, and the fastest is kept.
 * trial_ms (nullable, >= 32 floats) receives the medians (ms per step) in
 * candidate order and *n_trials their count. The choice is cached per process
 * by replica set (sizes, meshes, K, D, brick) and device: a later call for the
 * same set applies it without trials (*n_trials = 0). The trials advance the
 * simulation; the trajectory per bead is that of any other launch shape (the
 * storage order between sorts may differ). Synchronises the stream. */
hpf_status_t hpf_batch_tune(hpf_batch_t* batch, int32_t trial_steps, void* stream,
                            hpf_batch_config_t* chosen, float* trial_ms, int32_t* n_trials);
hpf_status_t hpf_batch_destroy(hpf_batch_t* batch);

/* HIP graphs around any sequence of library calls: capture what is enqueued
 * on `stream` (not the null stream) between begin and end, then replay it
 * with one launch. Buffers used during capture must outlive the graph. */
typedef struct hpf_graph hpf_graph_t;
hpf_status_t hpf_graph_begin(void* stream);
hpf_status_t hpf_graph_end(void* stream, hpf_graph_t** out);
hpf_status_t hpf_graph_launch(hpf_graph_t* graph, void* stream);
hpf_status_t hpf_graph_destroy(hpf_graph_t* graph);

/* Read (and optionally clear) the sticky device status bits of the current
 * device. Synchronises `stream`. flags is a HOST pointer. */
hpf_status_t hpf_get_device_status(uint32_t* flags, int32_t clear, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HPF_H */
