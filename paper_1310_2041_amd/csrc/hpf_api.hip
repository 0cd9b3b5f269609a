// Host side of the C ABI: argument checks, kernel-argument packing, dispatch.
// Every entry point validates on the host and enqueues on the caller's
// stream; nothing here allocates device memory.
//
// This file is the library's single translation unit: it includes the kernel
// sources below, so the device status word needs no relocatable device code.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "hpf_common.hpp"

namespace hpf {

__device__ uint32_t g_status = 0;

static bool mesh_ok(const hpf_mesh_t* m)
{
    if (!m)
        return false;
    for (int d = 0; d < 3; ++d) {
        if (!(m->L[d] > 0.0f) || !std::isfinite(m->L[d]))
            return false;
        if (m->M[d] < 3 || m->M[d] > (1 << 20))
            return false;
        if (!(m->s[d] > 0.0f) || !std::isfinite(m->s[d]))
            return false;
    }
    if ((int64_t)m->M[0] * m->M[1] * m->M[2] > (1LL << 34))
        return false;
    return std::isfinite(m->c_norm) && m->c_norm >= 0.0;
}

static MeshK mesh_k(const hpf_mesh_t* m)
{
    MeshK k;
    for (int d = 0; d < 3; ++d) {
        k.L[d] = m->L[d];
        k.halfL[d] = 0.5f * m->L[d];
        k.s[d] = m->s[d];
        k.M[d] = m->M[d];
    }
    k.nm = (int64_t)m->M[0] * m->M[1] * m->M[2];
    k.c_norm = m->c_norm;
    return k;
}

static bool box_ok(const float* box)
{
    if (!box)
        return false;
    for (int d = 0; d < 3; ++d)
        if (!(box[d] > 0.0f) || !std::isfinite(box[d]))
            return false;
    return true;
}

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Kernel form of a thermostat description; false for invalid parameters. A null
// description, or p = 0, is no thermostat (thr = 0).
struct ThermoK;
static bool thermo_k(const hpf_thermostat_t* t, int64_t N, ThermoK* out);

}  // namespace hpf

#include "hpf_scatter.hip"
#include "hpf_scatter_cells.hip"
#include "hpf_field.hip"
#include "hpf_particles.hip"
#include "hpf_sort.hip"

namespace hpf {

static bool thermo_k(const hpf_thermostat_t* t, int64_t N, ThermoK* out)
{
    *out = ThermoK{0u, 0.0f, 0u, 0u, nullptr, nullptr, 0u};
    if (!t || t->p == 0.0f)
        return true;
    if (!(t->p > 0.0f && t->p <= 1.0f) || !(t->kT > 0.0f) || !std::isfinite(t->kT) || !t->step ||
        (N > 0 && !t->tag))
        return false;
    // floor(p 2^24): exact, p * 2^24 is exact in double for a float p
    out->thr = t->p >= 1.0f ? (1u << 24) : (uint32_t)std::floor((double)t->p * 16777216.0);
    out->kT = t->kT;
    out->key0 = (uint32_t)t->seed;
    out->key1 = (uint32_t)(t->seed >> 32);
    out->step = t->step;
    out->tag = t->tag;
    out->tag_off = (uint32_t)t->tag_offset;
    return true;
}

// Device scratch of hpf_density_scatter_cells_static (its stray list and partial
// boxes) for callers that cannot allocate: a fixed array that every device holds
// while the library is loaded. In host code its name stands for a host-side shadow,
// not a device address; only its per-device address from hipGetSymbolAddress is
// passed to kernels.
static __device__ __align__(256) unsigned char scratch[HPF_STATIC_SCRATCH_BYTES];

// The device address of `scratch` on the current device, looked up on the first call
// made with that device current and kept per device.
static hpf_status_t static_scratch(char** out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return HPF_EHIP;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return HPF_EHIP;
        addr[dev] = p;
    }
    *out = static_cast<char*>(addr[dev]);
    return HPF_OK;
}

}  // namespace hpf

using namespace hpf;

extern "C" {

int32_t hpf_abi_version(void) { return HPF_ABI_VERSION; }

const char* hpf_status_string(hpf_status_t status)
{
    switch (status) {
    case HPF_OK: return "ok";
    case HPF_EINVAL: return "invalid argument";
    case HPF_EHIP: return "HIP runtime error";
    case HPF_ESPACE: return "workspace too small";
    case HPF_ETOOBIG: return "problem exceeds the library's fixed device scratch (HPF_STATIC_SCRATCH_BYTES)";
    default: return "unknown status";
    }
}

hpf_status_t hpf_mesh_make(const float* L, const int32_t* M, int64_t n_beads, hpf_mesh_t* out)
{
    if (!L || !M || !out || n_beads < 0)
        return HPF_EINVAL;
    hpf_mesh_t m{};
    int64_t nm = 1;
    for (int d = 0; d < 3; ++d) {
        if (!(L[d] > 0.0f) || !std::isfinite(L[d]) || M[d] < 3 || M[d] > (1 << 20))
            return HPF_EINVAL;
        m.L[d] = L[d];
        m.M[d] = M[d];
        m.s[d] = (float)((double)M[d] / (double)L[d]);
        nm *= M[d];
    }
    m.c_norm = n_beads > 0 ? (double)nm / (281474976710656.0 * (double)n_beads) : 0.0;
    *out = m;
    return HPF_OK;
}

hpf_status_t hpf_density_scatter(const float* R, const uint8_t* T, int64_t N, const hpf_mesh_t* mesh,
                                 int32_t K, uint64_t* counts, void* stream)
{
    if (N < 0 || !mesh_ok(mesh) || K < 1 || K > HPF_MAX_TYPES || !counts)
        return HPF_EINVAL;
    if (N > 0 && (!R || !T))
        return HPF_EINVAL;
    return launch_density_scatter(R, T, N, mesh_k(mesh), K, counts, as_stream(stream));
}

static bool scatter_cells_setup(int64_t N, const hpf_mesh_t* mesh, int32_t K, int32_t B, int32_t halo,
                                TileK* tk, size_t* stray_bytes, size_t* total_bytes)
{
    if (N < 0 || N > 0x7ffffff0LL || !mesh_ok(mesh) || K < 1 || K > HPF_MAX_TYPES)
        return false;
    if (B == 0)
        B = 8;
    if (B < 3 || B > kTcMaxB || halo < 0 || halo > kTcMaxHalo || halo >= B)
        return false;
    for (int d = 0; d < 3; ++d)
        if (mesh->M[d] < B + 1 + 2 * halo)
            return false;
    const int P = B + 1 + 2 * halo;
    if (scatter_cells_smem(K, P) > 160 * 1024)
        return false;
    int64_t nk = 1, nt = 1;
    for (int d = 0; d < 3; ++d) {
        tk->nb[d] = (mesh->M[d] + B - 1) / B;
        nk *= tk->nb[d];
        nt *= tk->nb[d];
    }
    if (nt > 0x7fffffffLL || nk > 0xfffffff0LL)
        return false;
    tk->m = mesh_k(mesh);
    tk->B = B;
    tk->h = halo;
    tk->P = P;
    tk->NK = (uint32_t)nk;
    tk->ntiles = nt;
    *stray_bytes = (sizeof(uint32_t) * (size_t)(N + 64) + 255) & ~(size_t)255;
    *total_bytes = *stray_bytes + scatter_cells_partials(nt, K, P);
    return true;
}

size_t hpf_scatter_workspace_bytes(int64_t N, const hpf_mesh_t* mesh, int32_t K, int32_t B, int32_t halo)
{
    TileK tk;
    size_t sb = 0, tb = 0;
    return scatter_cells_setup(N, mesh, K, B, halo, &tk, &sb, &tb) ? tb : 0;
}

hpf_status_t hpf_density_scatter_cells_static(const float* R, const uint8_t* T, int64_t N, const hpf_mesh_t* mesh,
                                              int32_t K, const uint32_t* cell_start, int32_t B, int32_t halo,
                                              uint64_t* counts, void* stream)
{
    TileK tk;
    size_t sb = 0, tb = 0;
    if (!counts || !cell_start || !scatter_cells_setup(N, mesh, K, B, halo, &tk, &sb, &tb))
        return HPF_EINVAL;
    if (N > 0 && (!R || !T))
        return HPF_EINVAL;
    if (tb > (size_t)HPF_STATIC_SCRATCH_BYTES)
        return HPF_ETOOBIG;
    char* w = nullptr;
    const hpf_status_t st = static_scratch(&w);
    if (st != HPF_OK)
        return st;
    // the stray counter at the head of the list is cleared by a kernel of the launch,
    // and every brick overwrites its whole partial box
    return launch_scatter_cells(R, T, N, tk, K, cell_start, counts, reinterpret_cast<uint32_t*>(w),
                                reinterpret_cast<unsigned long long*>(w + sb), as_stream(stream));
}

hpf_status_t hpf_density_scatter_cells(const float* R, const uint8_t* T, int64_t N, const hpf_mesh_t* mesh,
                                       int32_t K, const uint32_t* cell_start, int32_t B, int32_t halo,
                                       uint64_t* counts, void* work, size_t work_bytes, void* stream)
{
    TileK tk;
    size_t sb = 0, tb = 0;
    if (!counts || !cell_start || !scatter_cells_setup(N, mesh, K, B, halo, &tk, &sb, &tb))
        return HPF_EINVAL;
    if (N > 0 && (!R || !T))
        return HPF_EINVAL;
    if (!work || work_bytes < tb)
        return HPF_ESPACE;
    char* w = static_cast<char*>(work);
    return launch_scatter_cells(R, T, N, tk, K, cell_start, counts, reinterpret_cast<uint32_t*>(w),
                                reinterpret_cast<unsigned long long*>(w + sb), as_stream(stream));
}

// Field coefficients A = kT chi, 1/kappa and the energy scale; false for non-finite input.
static bool pot_params(const hpf_mesh_t* mesh, const hpf_field_t* field, PotK* p)
{
    const int K = field->K;
    *p = PotK{};
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            const double c = field->chi[a * K + b];
            if (!std::isfinite(c))
                return false;
            p->A[a * K + b] = field->kT * c;
        }
    if (!std::isfinite(field->kT) || !std::isfinite(field->inv_kappa))
        return false;
    p->inv_kappa = field->inv_kappa;
    p->rho0_dV = mesh->c_norm > 0.0 ? 1.0 / (mesh->c_norm * 281474976710656.0) : 0.0;
    return true;
}

hpf_status_t hpf_field_potential(uint64_t* counts, const hpf_mesh_t* mesh, const hpf_field_t* field,
                                 float* V, double* w_part, uint8_t* present, void* stream)
{
    if (!counts || !V || !mesh_ok(mesh) || !field || field->K < 1 || field->K > HPF_MAX_TYPES)
        return HPF_EINVAL;
    PotK p;
    if (!pot_params(mesh, field, &p))
        return HPF_EINVAL;
    return launch_field_potential(counts, mesh_k(mesh), field->K, p, V, w_part, present, as_stream(stream));
}

hpf_status_t hpf_field_potential_cells(uint64_t* counts, int64_t N, const hpf_mesh_t* mesh,
                                       const hpf_field_t* field, int32_t B, int32_t halo, const void* work,
                                       size_t work_bytes, float* V, double* w_part, uint8_t* present,
                                       void* stream)
{
    if (!counts || !V || !mesh_ok(mesh) || !field || field->K < 1 || field->K > HPF_MAX_TYPES)
        return HPF_EINVAL;
    TileK tk;
    size_t sb = 0, tb = 0;
    PotK p;
    if (!scatter_cells_setup(N, mesh, field->K, B, halo, &tk, &sb, &tb) || !pot_params(mesh, field, &p))
        return HPF_EINVAL;
    if (!work || work_bytes < tb)
        return HPF_ESPACE;
    const char* w = static_cast<const char*>(work);
    return launch_finish_potential(reinterpret_cast<const unsigned long long*>(w + sb), tk, field->K, p, counts, V,
                                   w_part, present, as_stream(stream));
}

hpf_status_t hpf_field_gradient(const float* V, const hpf_mesh_t* mesh, int32_t K, float* G,
                                const uint8_t* present, void* stream)
{
    if (!V || !G || !mesh_ok(mesh) || K < 1 || K > HPF_MAX_TYPES)
        return HPF_EINVAL;
    if ((mesh->M[0] + 63) / 64 > 65535 || mesh->M[2] > 65535)
        return HPF_EINVAL;
    return launch_field_gradient(V, mesh_k(mesh), K, G, present, as_stream(stream));
}

hpf_status_t hpf_force_gather(const float* R, const uint8_t* T, int64_t N, const hpf_mesh_t* mesh,
                              int32_t K, const float* G, float* F, void* stream)
{
    if (N < 0 || !mesh_ok(mesh) || K < 1 || K > HPF_MAX_TYPES || !G)
        return HPF_EINVAL;
    if (N > 0 && (!R || !T || !F))
        return HPF_EINVAL;
    return launch_force_gather(R, T, N, mesh_k(mesh), K, G, F, as_stream(stream));
}

hpf_status_t hpf_force_gather_staggered(const float* R, const uint8_t* T, int64_t N, const hpf_mesh_t* mesh,
                                        int32_t K, const float* V, float* F, void* stream)
{
    if (N < 0 || !mesh_ok(mesh) || K < 1 || K > HPF_MAX_TYPES || !V)
        return HPF_EINVAL;
    if (N > 0 && (!R || !T || !F))
        return HPF_EINVAL;
    return launch_force_gather_staggered(R, T, N, mesh_k(mesh), K, V, F, as_stream(stream));
}

hpf_status_t bond_forces(const float* R, int64_t N, const int32_t* bonds, int32_t D, float k, float r0,
                         const float* box, float* F, double* e_part, void* stream)
{
    if (N < 0 || N > 0x7fffffffLL || D < 0 || D > HPF_MAX_BONDS || !box_ok(box) ||
        !std::isfinite(k) || !std::isfinite(r0))
        return HPF_EINVAL;
    if (N > 0 && (!R || !F || (D > 0 && !bonds)))
        return HPF_EINVAL;
    BoxK b;
    for (int d = 0; d < 3; ++d) {
        b.L[d] = box[d];
        b.halfL[d] = 0.5f * box[d];
    }
    return launch_bond_forces(R, N, bonds, D, k, r0, b, F, e_part, as_stream(stream));
}

hpf_status_t angle_forces(const float* R, int64_t N, const int32_t* angles, int32_t A, int32_t ntypes,
                          const float* k, const float* theta0, const int32_t* form, const float* box, float* F,
                          double* e_part, void* stream)
{
    if (N < 0 || A < 0 || A > HPF_MAX_ANGLES || ntypes < 1 || ntypes > HPF_MAX_ANGLE_TYPES || !k || !theta0 ||
        !form || !box_ok(box))
        return HPF_EINVAL;
    if (N > 0 && (!R || !F || (A > 0 && !angles)))
        return HPF_EINVAL;
    AngleK ak{};
    ak.ntypes = ntypes;
    for (int t = 0; t < ntypes; ++t) {
        if (!std::isfinite(k[t]) || !std::isfinite(theta0[t]) || (form[t] != 0 && form[t] != 1))
            return HPF_EINVAL;
        ak.k[t] = k[t];
        ak.theta0[t] = theta0[t];
        ak.cos0[t] = (float)std::cos((double)theta0[t]);
        ak.form[t] = form[t];
    }
    BoxK b;
    for (int d = 0; d < 3; ++d) {
        b.L[d] = box[d];
        b.halfL[d] = 0.5f * box[d];
    }
    return launch_angle_forces(R, N, angles, A, ak, b, F, e_part, as_stream(stream));
}

hpf_status_t verlet_step(float* R, float* Vel, const float* F, const float* inv_mass, int64_t N, float dt,
                         const float* box, int32_t half, double* kin_part, void* stream)
{
    if (N < 0 || !box_ok(box) || !(dt > 0.0f) || !std::isfinite(dt) || (half != 1 && half != 2))
        return HPF_EINVAL;
    if (N > 0 && (!Vel || !F || (half == 1 && !R)))
        return HPF_EINVAL;
    BoxK b;
    for (int d = 0; d < 3; ++d) {
        b.L[d] = box[d];
        b.halfL[d] = 0.5f * box[d];
    }
    return launch_verlet(R, Vel, F, inv_mass, N, dt, b, half, kin_part, as_stream(stream));
}

hpf_status_t hpf_advance(const float* R, float* R_next, float* Vel, const uint8_t* T, int64_t N,
                         const hpf_mesh_t* mesh, int32_t K, const float* G, const int32_t* bonds, int32_t D,
                         float k, float r0, const float* box, const float* inv_mass, float dt, float* F_out,
                         double* e_part, double* kin_part, const hpf_thermostat_t* thermostat, void* stream)
{
    ThermoK th;
    if (!thermo_k(thermostat, N, &th))
        return HPF_EINVAL;
    if (N < 0 || N > 0x7fffffffLL || !mesh_ok(mesh) || K < 1 || K > HPF_MAX_TYPES || D < 0 ||
        D > HPF_MAX_BONDS || !box_ok(box) || !std::isfinite(k) || !std::isfinite(r0) || !(dt > 0.0f) ||
        !std::isfinite(dt))
        return HPF_EINVAL;
    if (N > 0 && (!R || !R_next || !Vel || !T || !G || (D > 0 && !bonds) || R == R_next))
        return HPF_EINVAL;
    BoxK b;
    for (int d = 0; d < 3; ++d) {
        b.L[d] = box[d];
        b.halfL[d] = 0.5f * box[d];
    }
    return launch_advance(R, R_next, Vel, T, N, mesh_k(mesh), K, G, bonds, D, k, r0, b, inv_mass, dt, F_out,
                          e_part, kin_part, th, as_stream(stream));
}

static bool advance_args_ok(int64_t N, const hpf_mesh_t* mesh, int32_t K, int32_t D, float k, float r0,
                            const float* box, float dt)
{
    return N >= 0 && N <= 0x7fffffffLL && mesh_ok(mesh) && K >= 1 && K <= HPF_MAX_TYPES && D >= 0 &&
           D <= HPF_MAX_BONDS && box_ok(box) && std::isfinite(k) && std::isfinite(r0) && dt > 0.0f &&
           std::isfinite(dt);
}

hpf_status_t hpf_advance_scatter(const float* R, float* R_next, float* Vel, const uint8_t* T, int64_t N,
                                 const hpf_mesh_t* mesh, int32_t K, const float* G, const int32_t* bonds,
                                 int32_t D, float k, float r0, const float* box, const float* inv_mass, float dt,
                                 const uint32_t* cell_start, int32_t B, int32_t halo, uint64_t* counts, void* work,
                                 size_t work_bytes, float* F_out, double* e_part, double* kin_part,
                                 const hpf_thermostat_t* thermostat, void* stream)
{
    TileK tk;
    ThermoK th;
    size_t sb = 0, tb = 0;
    if (!thermo_k(thermostat, N, &th))
        return HPF_EINVAL;
    if (!advance_args_ok(N, mesh, K, D, k, r0, box, dt) || !counts || !cell_start ||
        !scatter_cells_setup(N, mesh, K, B, halo, &tk, &sb, &tb))
        return HPF_EINVAL;
    if (N > 0 && (!R || !R_next || !Vel || !T || !G || (D > 0 && !bonds) || R == R_next))
        return HPF_EINVAL;
    if (!work || work_bytes < tb)
        return HPF_ESPACE;
    BoxK b;
    for (int d = 0; d < 3; ++d) {
        b.L[d] = box[d];
        b.halfL[d] = 0.5f * box[d];
    }
    char* w = static_cast<char*>(work);
    return launch_advance_scatter(R, R_next, Vel, T, N, tk, K, G, bonds, D, k, r0, b, inv_mass, dt, cell_start,
                                  reinterpret_cast<unsigned long long*>(w + sb),
                                  reinterpret_cast<unsigned long long*>(counts), F_out, e_part, kin_part, th,
                                  as_stream(stream));
}

hpf_status_t hpf_andersen(float* Vel, const float* inv_mass, int64_t N, const hpf_thermostat_t* thermostat,
                          double* kin_part, void* stream)
{
    ThermoK th;
    if (N < 0 || N > 0x7fffffffLL || !thermostat || !thermo_k(thermostat, N, &th) || (N > 0 && !Vel))
        return HPF_EINVAL;
    return launch_andersen(Vel, inv_mass, N, th, kin_part, as_stream(stream));
}

hpf_status_t hpf_density_finish_cells(uint64_t* counts, int64_t N, const hpf_mesh_t* mesh, int32_t K, int32_t B,
                                      int32_t halo, const void* work, size_t work_bytes, void* stream)
{
    TileK tk;
    size_t sb = 0, tb = 0;
    if (!counts || !scatter_cells_setup(N, mesh, K, B, halo, &tk, &sb, &tb))
        return HPF_EINVAL;
    if (!work || work_bytes < tb)
        return HPF_ESPACE;
    const char* w = static_cast<const char*>(work);
    return launch_scatter_finish(reinterpret_cast<const unsigned long long*>(w + sb), tk, K,
                                 reinterpret_cast<unsigned long long*>(counts), as_stream(stream));
}

hpf_status_t hpf_reduce_partials(const double* part, int32_t ncomp, double* out, void* stream)
{
    if (!part || !out || ncomp < 1 || ncomp > 8)
        return HPF_EINVAL;
    return launch_reduce_partials(part, ncomp, out, as_stream(stream));
}

size_t hpf_sort_workspace_bytes(int64_t N, const hpf_mesh_t* mesh, int32_t B)
{
    if (!mesh_ok(mesh))
        return 0;
    SortPlan plan;
    if (!sort_layout(N, mesh->M, B, nullptr, &plan))
        return 0;
    return plan.bytes;
}

hpf_status_t hpf_sort_by_cell(const hpf_mesh_t* mesh, int32_t B, int64_t N, const float* R_in,
                              const float* Vel_in, const uint8_t* T_in, const int32_t* tag_in,
                              const int32_t* bonds_in, int32_t D, float* R_out, float* Vel_out,
                              uint8_t* T_out, int32_t* tag_out, int32_t* bonds_out, uint32_t* cell_start,
                              void* work, size_t work_bytes, void* stream)
{
    if (!mesh_ok(mesh) || N < 0 || D < 0 || D > HPF_MAX_BONDS)
        return HPF_EINVAL;
    if (N > 0 && (!R_in || !T_in || !R_out || !T_out))
        return HPF_EINVAL;
    if (!Vel_in != !Vel_out || !tag_in != !tag_out || (N > 0 && D > 0 && (!bonds_in || !bonds_out)))
        return HPF_EINVAL;
    if (N > 0 && (R_in == R_out || (Vel_in && Vel_in == Vel_out) || T_in == T_out ||
                  (tag_in && tag_in == tag_out) || (D > 0 && bonds_in == bonds_out)))
        return HPF_EINVAL;
    SortK sk;
    SortPlan plan;
    if (!sort_layout(N, mesh->M, B, &sk, &plan))
        return HPF_EINVAL;
    if (!work || work_bytes < plan.bytes)
        return HPF_ESPACE;
    sk.m = mesh_k(mesh);
    return launch_sort(sk, plan, N, R_in, Vel_in, T_in, tag_in, bonds_in, D, R_out, Vel_out, T_out, tag_out,
                       bonds_out, cell_start, static_cast<char*>(work), as_stream(stream));
}

hpf_status_t hpf_resort_by_cell(const hpf_mesh_t* mesh, int32_t B, int64_t N, const float* R_in,
                                const float* Vel_in, const uint8_t* T_in, const int32_t* tag_in,
                                const int32_t* bonds_in, int32_t D, float* R_out, float* Vel_out, uint8_t* T_out,
                                int32_t* tag_out, int32_t* bonds_out, const uint32_t* cell_start_in,
                                uint32_t* cell_start_out, void* work, size_t work_bytes, void* stream)
{
    if (!mesh_ok(mesh) || N < 0 || D < 0 || D > HPF_MAX_BONDS || !cell_start_in || !cell_start_out ||
        cell_start_in == cell_start_out)
        return HPF_EINVAL;
    if (N > 0 && (!R_in || !T_in || !R_out || !T_out))
        return HPF_EINVAL;
    if (!Vel_in != !Vel_out || !tag_in != !tag_out || (N > 0 && D > 0 && (!bonds_in || !bonds_out)))
        return HPF_EINVAL;
    if (N > 0 && (R_in == R_out || (Vel_in && Vel_in == Vel_out) || T_in == T_out ||
                  (tag_in && tag_in == tag_out) || (D > 0 && bonds_in == bonds_out)))
        return HPF_EINVAL;
    SortK sk;
    SortPlan plan;
    if (!sort_layout(N, mesh->M, B, &sk, &plan))
        return HPF_EINVAL;
    if (!work || work_bytes < plan.bytes)
        return HPF_ESPACE;
    sk.m = mesh_k(mesh);
    return launch_resort(sk, plan, N, R_in, Vel_in, T_in, tag_in, bonds_in, D, R_out, Vel_out, T_out, tag_out,
                         bonds_out, cell_start_in, cell_start_out, static_cast<char*>(work), as_stream(stream));
}

hpf_status_t hpf_sort_angles(const hpf_mesh_t* mesh, int32_t B, int64_t N, const int32_t* angles_in, int32_t A,
                             int32_t* angles_out, const void* work, size_t work_bytes, void* stream)
{
    if (!mesh_ok(mesh) || N < 0 || A < 0 || A > HPF_MAX_ANGLES)
        return HPF_EINVAL;
    if (N > 0 && A > 0 && (!angles_in || !angles_out || angles_in == angles_out))
        return HPF_EINVAL;
    SortK sk;
    SortPlan plan;
    if (!sort_layout(N, mesh->M, B, &sk, &plan))
        return HPF_EINVAL;
    if (!work || work_bytes < plan.bytes)
        return HPF_ESPACE;
    return launch_sort_angles(plan, N, angles_in, A, angles_out, static_cast<const char*>(work),
                              as_stream(stream));
}

hpf_status_t hpf_get_device_status(uint32_t* flags, int32_t clear, void* stream)
{
    if (!flags)
        return HPF_EINVAL;
    if (hipStreamSynchronize(as_stream(stream)) != hipSuccess)
        return HPF_EHIP;
    uint32_t v = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_status), sizeof(v), 0, hipMemcpyDeviceToHost) != hipSuccess)
        return HPF_EHIP;
    if (clear) {
        const uint32_t z = 0;
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_status), &z, sizeof(z), 0, hipMemcpyHostToDevice) != hipSuccess)
            return HPF_EHIP;
    }
    *flags = v;
    return HPF_OK;
}

}  // extern "C"

#include "hpf_batch.hip"
