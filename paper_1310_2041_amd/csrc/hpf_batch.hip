// Batched replicas: many independent hPF-MD systems of uneven size and chi
// (a phase-diagram sweep) advanced by one set of kernel launches per phase.
//
// The replicas live in one concatenated set of bead arrays (replica r owns
// beads [off_r, off_r + N_r); bond-table entries are global indices) and one
// concatenated set of meshes (replica r's [K][M_r^3] block at K * moff_r).
// Cell keys of replica r are offset by key_base_r, so one counting sort over
// the concatenated key space sorts every replica inside its own bead range,
// and the single-system sort kernels are reused unchanged. Every other phase
// walks a host-built work list of (replica, range) items, one workgroup per
// item, with each XCD taking one contiguous run of items (so neighbouring
// ranges of a replica share that XCD's L2), and calls the same device functions as the single-system kernels, so
// each replica's beads follow exactly the trajectory they would follow alone.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "hpf_common.hpp"
#include "hpf_thermo.hpp"

namespace hpf {

struct RepK {
    MeshK m;
    BoxK box;
    PotK p;
    int64_t bead_off, N;
    int64_t moff;          // first mesh point of the replica in the concatenated meshes
    uint32_t key_base, NK;
    int32_t nb[3];
    int64_t brick_off;     // first brick of the replica in the concatenated brick numbering
    int64_t nbricks;
    float kT;              // the replica's temperature (its thermostat's bath)
};

struct ItemK {
    int32_t rep;
    int32_t aux;
    int64_t begin, end;
};

constexpr int kBThreads = 256;
constexpr int kASThreadsBatch = 512;

__device__ __forceinline__ TileK tile_of(const RepK& r, int B, int h)
{
    TileK t;
    t.m = r.m;
    t.B = B;
    t.h = h;
    t.P = B + 1 + 2 * h;
    t.nb[0] = r.nb[0];
    t.nb[1] = r.nb[1];
    t.nb[2] = r.nb[2];
    t.NK = r.NK;
    t.ntiles = r.nbricks;
    return t;
}

// ------------------------------------------------------------- cell scatter

__global__ __launch_bounds__(kTcThreads) void k_batch_scatter_bricks(const RepK* __restrict__ reps,
                                                                     const ItemK* __restrict__ items,
                                                                     int B, int h, int K,
                                                                     const float3* __restrict__ R,
                                                                     const uint8_t* __restrict__ T,
                                                                     const uint32_t* __restrict__ cell_start,
                                                                     unsigned long long* __restrict__ partials,
                                                                     uint32_t* __restrict__ strays)
{
    const int64_t li = xcd_block(blockIdx.x, gridDim.x);
    const ItemK it = items[li];
    const RepK& rp = reps[it.rep];
    const TileK tk = tile_of(rp, B, h);
    const int P = tk.P;
    scatter_brick_body(R, T, K, tk, cell_start + rp.key_base, it.begin,
                       partials + (rp.brick_off + it.begin) * (int64_t)K * P * P * P, strays);
}

template <bool kAdd>
__global__ __launch_bounds__(kSumThreads) void k_batch_scatter_sum(const RepK* __restrict__ reps,
                                                           const ItemK* __restrict__ items, int B, int h,
                                                           int K,
                                                           const unsigned long long* __restrict__ partials,
                                                           unsigned long long* __restrict__ counts)
{
    const int64_t li = xcd_block(blockIdx.x, gridDim.x);
    const ItemK it = items[li];
    const RepK& rp = reps[it.rep];
    const TileK tk = tile_of(rp, B, h);
    const int P = tk.P;
    scatter_sum_body<kAdd>(partials + rp.brick_off * (int64_t)K * P * P * P, tk, K, it.begin,
                     counts + (int64_t)K * rp.moff);
}

__device__ __forceinline__ int find_rep(const RepK* reps, int nrep, int64_t p)
{
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (reps[mid].bead_off <= p)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Sort key of bead i of the batch: its replica's key base plus its brick (or
// the replica's "cannot be binned" key).
struct RepKeyer {
    const RepK* reps;
    int nrep;
    int B;
    const float3* R;
    __device__ __forceinline__ uint32_t operator()(int32_t i) const
    {
        // Lanes of a wave nearly always hold beads of one replica: search once for the
        // first active lane (a uniform search), and per lane only outside its range.
        const int32_t i0 = __builtin_amdgcn_readfirstlane(i);
        int r = find_rep(reps, nrep, i0);
        if (!(i >= reps[r].bead_off && i < reps[r].bead_off + reps[r].N))
            r = find_rep(reps, nrep, i);
        const RepK& rp = reps[r];
        BeadCell b;
        return rp.key_base + (bead_cell(R[i], rp.m, b) ? brick_of(b.c[0], b.c[1], b.c[2], B, rp.nb) : rp.NK);
    }
};

// Strays of all replicas (global indices in one list) and each replica's
// beads that the sort could not bin, with global atomics.
__global__ __launch_bounds__(kTcThreads) void k_batch_scatter_strays(const RepK* __restrict__ reps, int nrep,
                                                                     int K, const float3* __restrict__ R,
                                                                     const uint8_t* __restrict__ T,
                                                                     const uint32_t* __restrict__ cell_start,
                                                                     const uint32_t* __restrict__ strays,
                                                                     unsigned long long* __restrict__ counts)
{
    const int64_t nstray = strays[0];
    bool bad = false;
    for (int64_t j = (int64_t)blockIdx.x * kTcThreads + threadIdx.x; j < nstray;
         j += (int64_t)gridDim.x * kTcThreads) {
        const int64_t p = strays[1 + j];
        const RepK& rp = reps[find_rep(reps, nrep, p)];
        bad |= !deposit_global(R[p], T[p], K, rp.m, counts + (int64_t)K * rp.moff);
    }
    // unbinned tails: replica r's beads with key key_base_r + NK_r
    for (int r = blockIdx.x; r < nrep; r += gridDim.x) {
        const RepK& rp = reps[r];
        const int64_t a = cell_start[rp.key_base + rp.NK], b = cell_start[rp.key_base + rp.NK + 1];
        for (int64_t p = a + threadIdx.x; p < b; p += kTcThreads)
            bad |= !deposit_global(R[p], T[p], K, rp.m, counts + (int64_t)K * rp.moff);
    }
    if (bad)
        raise_flag(HPF_FLAG_BAD_BEAD);
}

// ---------------------------------------------------------- potential, grad

template <int K>
__global__ __launch_bounds__(kPotThreads) void k_batch_potential(const RepK* __restrict__ reps,
                                                                 const ItemK* __restrict__ items,
                                                                 unsigned long long* __restrict__ counts,
                                                                 float* __restrict__ V,
                                                                 double* __restrict__ w_part)
{
    __shared__ double scratch[kPotThreads / kWave];
    const int64_t li = xcd_block(blockIdx.x, gridDim.x);
    const ItemK it = items[li];
    const RepK& rp = reps[it.rep];
    double wsum = 0.0;
    bool over = false;
    unsigned long long* c = counts + (int64_t)K * rp.moff;
    float* v = V + (int64_t)K * rp.moff;
    for (int64_t q = it.begin + threadIdx.x; q < it.end; q += kPotThreads)
        wsum += potential_point<K>(c, v, rp.m.nm, q, rp.m.c_norm, rp.p, over, nullptr);
    if (over)
        raise_flag(HPF_FLAG_OVERFLOW);
    if (w_part) {
        const double s = block_sum(wsum, scratch);
        if (threadIdx.x == 0)
            w_part[li] = s * rp.p.rho0_dV;
    }
}

// The finish of the fused deposit and the potential in one pass, one
// workgroup per brick item: the covering boxes are summed onto the counts held
// at each point (the strays), V follows and the counts are cleared; the
// workgroup's field-energy term goes to slot li.
template <int K>
__global__ __launch_bounds__(kFPThreads) void k_batch_finish_potential(const RepK* __restrict__ reps,
                                                                       const ItemK* __restrict__ items, int B,
                                                                       int h,
                                                                       const unsigned long long* __restrict__ partials,
                                                                       unsigned long long* __restrict__ counts,
                                                                       float* __restrict__ V,
                                                                       double* __restrict__ w_part)
{
    __shared__ Cover cov[3][kTcMaxB];
    __shared__ double scratch[kFPThreads / kWave];
    const int64_t li = xcd_block(blockIdx.x, gridDim.x);
    const ItemK it = items[li];
    const RepK& rp = reps[it.rep];
    const TileK tk = tile_of(rp, B, h);
    const int P = tk.P;
    bool over = false;
    const double wsum = finish_potential_brick<K>(cov, partials + rp.brick_off * (int64_t)K * P * P * P, tk, rp.p,
                                                  counts + (int64_t)K * rp.moff, V + (int64_t)K * rp.moff,
                                                  it.begin, over, nullptr);
    if (over)
        raise_flag(HPF_FLAG_OVERFLOW);
    if (w_part) {
        const double s = block_sum(wsum, scratch);
        if (threadIdx.x == 0)
            w_part[li] = s * rp.p.rho0_dV;
    }
}

// one workgroup per (replica, z plane)
__global__ __launch_bounds__(256) void k_batch_gradient(const RepK* __restrict__ reps,
                                                        const ItemK* __restrict__ items, int K,
                                                        const float* __restrict__ V,
                                                        float3* __restrict__ G)
{
    const int64_t li = xcd_block(blockIdx.x, gridDim.x);
    const ItemK it = items[li];
    const RepK& rp = reps[it.rep];
    const int Mx = rp.m.M[0], My = rp.m.M[1];
    const int z = (int)it.begin;
    for (int e = threadIdx.x; e < Mx * My; e += 256)
        gradient_point(V + (int64_t)K * rp.moff, rp.m, K, e % Mx, e / Mx, z, G + (int64_t)K * rp.moff);
}

// ------------------------------------------------------------------ advance

template <bool kR0Zero, bool kThermo>
__global__ __launch_bounds__(kPThreads) void k_batch_advance(const RepK* __restrict__ reps,
                                                             const ItemK* __restrict__ items, int K,
                                                             const float3* __restrict__ R,
                                                             float3* __restrict__ R_next,
                                                             float3* __restrict__ Vel,
                                                             const uint8_t* __restrict__ T, int64_t Ntot,
                                                             const float3* __restrict__ G,
                                                             const int32_t* __restrict__ bonds, int D, float k,
                                                             float r0, float dt,
                                                             double* __restrict__ e_part,
                                                             double* __restrict__ kin_part, int nslot, ThermoK th)
{
    __shared__ double scratch[kPThreads / kWave];
    const int64_t li = xcd_block(blockIdx.x, gridDim.x);
    const ItemK it = items[li];
    const RepK& rp = reps[it.rep];
    th.kT = rp.kT;
    const uint64_t tstep = thermo_step(th);
    const float3* Gr = G + (int64_t)K * rp.moff;
    const float hdt = 0.5f * dt;
    KinAcc acc;
    double e = 0.0;
    bool bad_bead = false, bad_bond = false, nonfinite = false;
    for (int64_t i = it.begin + threadIdx.x; i < it.end; i += kPThreads)
        advance_bead<kR0Zero, kThermo>(i, R, R_next, Vel, T, Ntot, rp.m, K, Gr, bonds, D, k, r0, rp.box, nullptr,
                              dt, hdt, nullptr, acc, e, bad_bead, bad_bond, nonfinite, th, tstep);
    if (bad_bead)
        raise_flag(HPF_FLAG_BAD_BEAD);
    if (bad_bond)
        raise_flag(HPF_FLAG_BAD_BOND);
    if (nonfinite)
        raise_flag(HPF_FLAG_NONFINITE);
    if (e_part) {
        const double s = block_sum(e, scratch);
        if (threadIdx.x == 0)
            e_part[li] = s;
    }
    if (kin_part)
        acc.store_rows(kin_part, nslot, li, scratch);
}

// The fused pass with the density deposit of the new positions (as
// k_advance_scatter), one workgroup per (replica, brick) item of the last
// sort; a replica's last item (brick == NK) holds the beads the sort could
// not bin, deposited with global atomics. The energy partials go to the
// item's slot. kNT as in k_advance_scatter, chosen on the bytes of the whole batch.
template <bool kR0Zero, bool kPipe, bool kThermo, bool kNT>
__global__ __launch_bounds__(kASThreadsBatch) void k_batch_advance_scatter(
    const RepK* __restrict__ reps, const ItemK* __restrict__ items, int B, int h, int K,
    const float3* __restrict__ R, float3* __restrict__ R_next, float3* __restrict__ Vel,
    const uint8_t* __restrict__ T, int64_t Ntot, const float3* __restrict__ G, const int32_t* __restrict__ bonds,
    int D, float k, float r0, float dt, const uint32_t* __restrict__ cell_start,
    unsigned long long* __restrict__ partials, unsigned long long* __restrict__ counts,
    double* __restrict__ e_part, double* __restrict__ kin_part, int nslot, ThermoK th)
{
    extern __shared__ unsigned long long dbox[];
    __shared__ double scratch[kASThreadsBatch / kWave];
    const int64_t li = xcd_block(blockIdx.x, gridDim.x);
    const ItemK it = items[li];
    const RepK& rp = reps[it.rep];
    th.kT = rp.kT;
    const uint64_t tstep = thermo_step(th);
    const MeshK& m = rp.m;
    const float3* Gr = G + (int64_t)K * rp.moff;
    unsigned long long* cr = counts + (int64_t)K * rp.moff;
    const int P = B + 1 + 2 * h, P3 = P * P * P, nbox = K * P3;
    const int64_t brick = it.begin;
    const float hdt = 0.5f * dt;
    KinAcc acc;
    double e = 0.0;
    bool bad_bead = false, bad_bond = false, nonfinite = false;
    const uint32_t* cs = cell_start + rp.key_base;
    if (brick < rp.NK) {
        const int bx = (int)(brick % rp.nb[0]);
        const int by = (int)((brick / rp.nb[0]) % rp.nb[1]);
        const int bz = (int)(brick / ((int64_t)rp.nb[0] * rp.nb[1]));
        const int x0 = bx * B, y0 = by * B, z0 = bz * B;
        const int ox = min(B, m.M[0] - x0), oy = min(B, m.M[1] - y0), oz = min(B, m.M[2] - z0);
        for (int q = threadIdx.x; q < nbox; q += kASThreadsBatch)
            dbox[q] = 0ull;
        __syncthreads();
        const int64_t first = cs[brick], last = min((int64_t)cs[brick + 1], Ntot);
        if (kPipe) {
            // software-pipelined as in k_advance_scatter (the table has at most kPreBonds rows)
            int64_t i = first + threadIdx.x;
            BeadIn cur;
            if (i < last)
                bead_fetch<kThermo, kNT>(cur, i, R, Vel, T, bonds, D, Ntot, nullptr, th);
            for (; i < last; i += kASThreadsBatch) {
                BeadLoads L;
                if constexpr (kNT)
                    __builtin_amdgcn_s_setprio(1);
                bead_issue(L, cur, i, m, K, Gr, R, Ntot);
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (kNT)
                    __builtin_amdgcn_s_setprio(0);
                BeadIn nxt;
                bead_fetch<kThermo, kNT>(nxt, min(i + kASThreadsBatch, last - 1), R, Vel, T, bonds, D, Ntot, nullptr,
                                    th);
                __builtin_amdgcn_sched_barrier(0);
                const float3 rn = bead_finish<kR0Zero, kThermo, kNT>(i, cur, L, R_next, Vel, Ntot, D, k, r0, rp.box, dt,
                                                                hdt,
                                                       nullptr, acc, e, bad_bead, bad_bond, nonfinite, th, tstep);
                const int t = cur.t;
                BeadCell bc;
                int lx, ly, lz;
                if (bead_cell(rn, m, bc) && t < K && brick_box_cell(bc, m, x0, y0, z0, ox, oy, oz, h, lx, ly, lz))
                    box_deposit(dbox, P, t, lx, ly, lz, bc);
                else
                    bad_bead |= !deposit_global(rn, t, K, m, cr);
                cur = nxt;
            }
        } else {
            for (int64_t i = first + threadIdx.x; i < last; i += kASThreadsBatch) {
                const float3 rn = advance_bead<kR0Zero, kThermo>(i, R, R_next, Vel, T, Ntot, m, K, Gr, bonds, D, k,
                                                                 r0, rp.box, nullptr, dt, hdt, nullptr, acc, e, bad_bead, bad_bond,
                                                        nonfinite, th, tstep);
                const int t = T[i];
                BeadCell bc;
                int lx, ly, lz;
                if (bead_cell(rn, m, bc) && t < K && brick_box_cell(bc, m, x0, y0, z0, ox, oy, oz, h, lx, ly, lz))
                    box_deposit(dbox, P, t, lx, ly, lz, bc);
                else
                    bad_bead |= !deposit_global(rn, t, K, m, cr);
            }
        }
        __syncthreads();
        unsigned long long* out = partials + (rp.brick_off + brick) * (int64_t)nbox;
        for (int q = threadIdx.x; q < nbox; q += kASThreadsBatch)
            store_hint<kNT>(out + q, dbox[q]);
    } else {
        const int64_t first = cs[rp.NK], last = min((int64_t)cs[rp.NK + 1], Ntot);
        for (int64_t i = first + threadIdx.x; i < last; i += kASThreadsBatch) {
            const float3 rn = advance_bead<kR0Zero, kThermo>(i, R, R_next, Vel, T, Ntot, m, K, Gr, bonds, D, k, r0,
                                                             rp.box,
                                                    nullptr, dt, hdt, nullptr, acc, e, bad_bead, bad_bond, nonfinite,
                                                    th, tstep);
            bad_bead |= !deposit_global(rn, T[i], K, m, cr);
        }
    }
    if (bad_bead)
        raise_flag(HPF_FLAG_BAD_BEAD);
    if (bad_bond)
        raise_flag(HPF_FLAG_BAD_BOND);
    if (nonfinite)
        raise_flag(HPF_FLAG_NONFINITE);
    if (e_part) {
        const double s = block_sum(e, scratch);
        if (threadIdx.x == 0)
            e_part[li] = s;
    }
    if (kin_part)
        acc.store_rows(kin_part, nslot, li, scratch);
}

// per replica: energies {KE, E_bond, W, E_tot, Px, Py, Pz, 0} from the item
// partials, each summed in item order by one lane
__global__ __launch_bounds__(64) void k_batch_reduce(const int64_t* __restrict__ bead_items,
                                                     const int64_t* __restrict__ mesh_items,
                                                     const double* __restrict__ w_part,
                                                     const double* __restrict__ e_part,
                                                     const double* __restrict__ kin_part, int nslot,
                                                     double* __restrict__ out)
{
    __shared__ double sums[6];
    const int r = blockIdx.x;
    const int c = threadIdx.x;
    if (c < 6) {
        double s = 0.0;
        if (c == 0) {
            for (int64_t i = mesh_items[r]; i < mesh_items[r + 1]; ++i)
                s += w_part[i];
        } else if (c == 1) {
            for (int64_t i = bead_items[r]; i < bead_items[r + 1]; ++i)
                s += e_part[i];
        } else {
            const double* row = kin_part + (int64_t)(c - 2) * nslot;
            for (int64_t i = bead_items[r]; i < bead_items[r + 1]; ++i)
                s += row[i];
        }
        sums[c] = s;
    }
    __syncthreads();
    if (c == 0) {
        double* o = out + (int64_t)r * 8;
        o[0] = sums[2];                    // KE
        o[1] = sums[1];                    // E_bond
        o[2] = sums[0];                    // W
        o[3] = sums[2] + sums[1] + sums[0];
        o[4] = sums[3];
        o[5] = sums[4];
        o[6] = sums[5];
        o[7] = 0.0;
    }
}

}  // namespace hpf

// ======================================================================
// Host side: replica table, work lists, workspace, launches, autotuner.
// ======================================================================

namespace hpf {

// The batch's device time level (a kernel, so that captured graphs advance it).
__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }
__global__ void k_add_i64(int64_t* p, int64_t v) { *p += v; }

// prime: forces at x_0, energies with v_0, then the first half step
template <bool kR0Zero>
__global__ __launch_bounds__(kPThreads) void k_batch_prime(const RepK* __restrict__ reps,
                                                           const ItemK* __restrict__ items, int K,
                                                           const float3* __restrict__ R,
                                                           float3* __restrict__ R_next,
                                                           float3* __restrict__ Vel,
                                                           const uint8_t* __restrict__ T, int64_t Ntot,
                                                           const float3* __restrict__ G,
                                                           const int32_t* __restrict__ bonds, int D, float k,
                                                           float r0, float dt, double* __restrict__ e_part,
                                                           double* __restrict__ kin_part, int nslot)
{
    __shared__ double scratch[kPThreads / kWave];
    const int64_t li = xcd_block(blockIdx.x, gridDim.x);
    const ItemK it = items[li];
    const RepK& rp = reps[it.rep];
    const float3* Gr = G + (int64_t)K * rp.moff;
    const float hdt = 0.5f * dt;
    KinAcc acc;
    double e = 0.0;
    bool bad_bead = false, bad_bond = false, nonfinite = false;
    for (int64_t i = it.begin + threadIdx.x; i < it.end; i += kPThreads) {
        float3 r = R[i];
        float3 ff;
        bad_bead |= !field_force(r, T[i], rp.m, K, Gr, ff);
        float ei;
        const float3 fb = bond_sum<kR0Zero>(i, r, R, Ntot, bonds, D, k, r0, rp.box, ei, bad_bond);
        float3 f = make_float3(ff.x, ff.y, ff.z);
        f.x += fb.x;
        f.y += fb.y;
        f.z += fb.z;
        e += 0.5 * (double)ei;
        float3 v = Vel[i];
        acc.add(v, 1.0f);
        kick(v, f, 1.0f, hdt);
        drift(r, v, dt, rp.box);
        nonfinite |= !(finite3(r) && finite3(v));
        Vel[i] = v;
        R_next[i] = r;
    }
    if (bad_bead)
        raise_flag(HPF_FLAG_BAD_BEAD);
    if (bad_bond)
        raise_flag(HPF_FLAG_BAD_BOND);
    if (nonfinite)
        raise_flag(HPF_FLAG_NONFINITE);
    if (e_part) {
        const double s = block_sum(e, scratch);
        if (threadIdx.x == 0)
            e_part[li] = s;
    }
    if (kin_part)
        acc.store_rows(kin_part, nslot, li, scratch);
}

constexpr int kMinBeadChunk = 512;
constexpr int kMinMeshChunk = 2048;

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
    int64_t Ntot = 0, nm_tot = 0, bricks_tot = 0;
    uint32_t NKT = 0;                    // keys of all replicas, invalid buckets included
    int64_t max_bead_items = 0, max_mesh_items = 0, max_planes = 0;
    int64_t nslot = 0;                   // energy partial slots (one per bead or fused item)
    size_t off_reps, off_bead_items, off_brick_items, off_adv_items, off_mesh_items, off_plane_items, off_bead_ioff,
        off_adv_ioff, off_mesh_ioff, off_brick_ioff, off_sort, off_start, off_strays, off_partials, off_wpart, off_epart, off_kpart, off_energy,
        off_tstep, total;
    SortPlan sort;
};

static bool batch_layout(const hpf_replica_t* reps, int nrep, const hpf_batch_config_t* cfg, BatchLayout* L)
{
    if (!reps || nrep < 1 || !cfg || cfg->K < 1 || cfg->K > HPF_MAX_TYPES || cfg->D < 0 ||
        cfg->D > HPF_MAX_BONDS)
        return false;
    const int B = cfg->brick == 0 ? 8 : cfg->brick;
    if (B < 3 || B > kTcMaxB)
        return false;
    const int Pmax = B + 1 + 2 * kTcMaxHalo;
    int64_t nkt = 0, expect_off = 0;
    for (int r = 0; r < nrep; ++r) {
        const hpf_replica_t& q = reps[r];
        if (q.n_beads < 0 || q.bead_offset != expect_off)
            return false;
        expect_off += q.n_beads;
        int64_t nk = 1, nbr = 1, nm = 1;
        for (int d = 0; d < 3; ++d) {
            if (!(q.L[d] > 0.0f) || q.M[d] < B + 1 + 2 * kTcMaxHalo || q.M[d] > 4096)
                return false;
            const int nb = (q.M[d] + B - 1) / B;
            nk *= nb;
            nbr *= nb;
            nm *= q.M[d];
        }
        nkt += nk + 1;
        L->bricks_tot += nbr;
        L->nm_tot += nm;
        L->max_bead_items += (q.n_beads + kMinBeadChunk - 1) / kMinBeadChunk;
        L->max_mesh_items += (nm + kMinMeshChunk - 1) / kMinMeshChunk;
        L->max_planes += q.M[2];
    }
    L->Ntot = expect_off;
    if (L->Ntot > 0x7ffffff0LL || !sort_plan(L->Ntot, nkt, &L->sort))
        return false;
    L->NKT = (uint32_t)nkt;
    const int64_t N1 = L->Ntot > 0 ? L->Ntot : 1;
    const int64_t nscan = nkt + 1;
    size_t o = 0;
    L->off_reps = o; o += al256(sizeof(RepK) * nrep);
    L->off_bead_items = o; o += al256(sizeof(ItemK) * (L->max_bead_items + 1));
    L->off_brick_items = o; o += al256(sizeof(ItemK) * (L->bricks_tot + 1));
    L->off_adv_items = o; o += al256(sizeof(ItemK) * (L->bricks_tot + nrep + 1));
    L->off_mesh_items = o; o += al256(sizeof(ItemK) * (L->max_mesh_items + 1));
    L->off_plane_items = o; o += al256(sizeof(ItemK) * (L->max_planes + 1));
    L->off_bead_ioff = o; o += al256(sizeof(int64_t) * (nrep + 1));
    L->off_adv_ioff = o; o += al256(sizeof(int64_t) * (nrep + 1));
    L->off_mesh_ioff = o; o += al256(sizeof(int64_t) * (nrep + 1));
    L->off_brick_ioff = o; o += al256(sizeof(int64_t) * (nrep + 1));
    L->off_sort = o; o += al256(L->sort.bytes);
    L->off_start = o; o += al256(sizeof(uint32_t) * (nscan + 1));
    L->off_strays = o; o += al256(sizeof(uint32_t) * (N1 + 64));
    L->off_partials = o; o += al256(sizeof(unsigned long long) * L->bricks_tot * cfg->K * Pmax * Pmax * Pmax);
    L->off_wpart = o; o += al256(sizeof(double) * (std::max(L->max_mesh_items, L->bricks_tot) + 1));
    L->nslot = std::max<int64_t>(L->max_bead_items, L->bricks_tot + nrep) + 1;
    L->off_epart = o; o += al256(sizeof(double) * L->nslot);
    L->off_kpart = o; o += al256(sizeof(double) * 4 * L->nslot);
    L->off_energy = o; o += al256(sizeof(double) * 8 * nrep);
    L->off_tstep = o; o += al256(sizeof(int64_t));
    L->total = o;
    return true;
}

}  // namespace hpf

struct hpf_batch {
    int nrep = 0;
    hpf_batch_config_t cfg{};
    hpf::BatchLayout L;
    std::vector<hpf::RepK> reps;
    std::vector<hpf_replica_t> desc;
    char* work = nullptr;
    hpf_batch_buffers_t buf{};
    int rcur = 0;        // current position buffer
    int scur = 0;        // current velocity / type / tag / bond buffer
    int64_t steps_done = 0;
    int64_t n_bead_items = 0, n_brick_items = 0, n_adv_items = 0, n_mesh_items = 0, n_planes = 0;
    bool pending = false;  // partial boxes + counts hold the deposit of the current positions
    bool w_bricks = false; // the last field pass left its W partials per brick item (else per mesh item)
    template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(work + off); }
};

namespace hpf {

static hpf_status_t batch_build_items(hpf_batch* b)
{
    const hpf_batch_config_t& c = b->cfg;
    std::vector<ItemK> bead, brick, adv, mesh, plane;
    std::vector<int64_t> bead_off(b->nrep + 1), adv_off(b->nrep + 1), mesh_off(b->nrep + 1),
        brick_off(b->nrep + 1);
    for (int r = 0; r < b->nrep; ++r) {
        const RepK& rp = b->reps[r];
        bead_off[r] = (int64_t)bead.size();
        for (int64_t s = 0; s < rp.N; s += c.bead_chunk)
            bead.push_back({r, 0, rp.bead_off + s, rp.bead_off + std::min<int64_t>(rp.N, s + c.bead_chunk)});
        mesh_off[r] = (int64_t)mesh.size();
        for (int64_t s = 0; s < rp.m.nm; s += c.mesh_chunk)
            mesh.push_back({r, 0, s, std::min<int64_t>(rp.m.nm, s + c.mesh_chunk)});
        brick_off[r] = (int64_t)brick.size();
        for (int64_t k = 0; k < rp.nbricks; ++k)
            brick.push_back({r, 0, k, k + 1});
        adv_off[r] = (int64_t)adv.size();
        for (int64_t k = 0; k <= rp.nbricks; ++k)          // the last item: beads that were not binned
            adv.push_back({r, 0, k, k + 1});
        for (int z = 0; z < rp.m.M[2]; ++z)
            plane.push_back({r, 0, z, z + 1});
    }
    bead_off[b->nrep] = (int64_t)bead.size();
    adv_off[b->nrep] = (int64_t)adv.size();
    mesh_off[b->nrep] = (int64_t)mesh.size();
    brick_off[b->nrep] = (int64_t)brick.size();
    if ((int64_t)bead.size() > b->L.max_bead_items || (int64_t)mesh.size() > b->L.max_mesh_items)
        return HPF_EINVAL;
    b->n_bead_items = (int64_t)bead.size();
    b->n_brick_items = (int64_t)brick.size();
    b->n_adv_items = (int64_t)adv.size();
    b->n_mesh_items = (int64_t)mesh.size();
    b->pending = false;                 // launch shapes may change the deposit boxes
    b->n_planes = (int64_t)plane.size();
    auto up = [&](size_t off, const void* src, size_t bytes) {
        return bytes == 0 || hipMemcpy(b->work + off, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(b->L.off_bead_items, bead.data(), sizeof(ItemK) * bead.size()) ||
        !up(b->L.off_brick_items, brick.data(), sizeof(ItemK) * brick.size()) ||
        !up(b->L.off_adv_items, adv.data(), sizeof(ItemK) * adv.size()) ||
        !up(b->L.off_adv_ioff, adv_off.data(), sizeof(int64_t) * adv_off.size()) ||
        !up(b->L.off_mesh_items, mesh.data(), sizeof(ItemK) * mesh.size()) ||
        !up(b->L.off_plane_items, plane.data(), sizeof(ItemK) * plane.size()) ||
        !up(b->L.off_bead_ioff, bead_off.data(), sizeof(int64_t) * bead_off.size()) ||
        !up(b->L.off_mesh_ioff, mesh_off.data(), sizeof(int64_t) * mesh_off.size()) ||
        !up(b->L.off_brick_ioff, brick_off.data(), sizeof(int64_t) * brick_off.size()))
        return HPF_EHIP;
    return HPF_OK;
}

static hpf_status_t batch_sort(hpf_batch* b, hipStream_t s)
{
    const BatchLayout& L = b->L;
    const int o = b->scur, n = 1 - b->scur;
    RepKeyer keyer{b->at<RepK>(L.off_reps), b->nrep, b->cfg.brick,
                   reinterpret_cast<const float3*>(b->buf.R[b->rcur])};
    const hpf_status_t st =
        run_sort(L.sort, keyer, L.Ntot, b->buf.R[b->rcur], b->buf.Vel[o], b->buf.T[o], b->buf.tag[o],
                 b->cfg.D > 0 ? b->buf.bonds[o] : nullptr, b->cfg.D, b->buf.R[1 - b->rcur], b->buf.Vel[n],
                 b->buf.T[n], b->buf.tag[n], b->cfg.D > 0 ? b->buf.bonds[n] : nullptr, b->at<uint32_t>(L.off_start),
                 b->work + L.off_sort, s);
    b->rcur = 1 - b->rcur;
    b->scur = n;
    return st;
}

// The potential over the mesh items, from counts that are complete.
static hpf_status_t batch_potential(hpf_batch* b, int K, unsigned long long* counts, double* w, hipStream_t s)
{
    const RepK* reps = b->at<RepK>(b->L.off_reps);
    const dim3 gm((unsigned)b->n_mesh_items), bm(kPotThreads);
    const ItemK* mi = b->at<ItemK>(b->L.off_mesh_items);
    float* V = b->buf.V;
    switch (K) {
    case 1: hipLaunchKernelGGL(k_batch_potential<1>, gm, bm, 0, s, reps, mi, counts, V, w); break;
    case 2: hipLaunchKernelGGL(k_batch_potential<2>, gm, bm, 0, s, reps, mi, counts, V, w); break;
    case 3: hipLaunchKernelGGL(k_batch_potential<3>, gm, bm, 0, s, reps, mi, counts, V, w); break;
    case 4: hipLaunchKernelGGL(k_batch_potential<4>, gm, bm, 0, s, reps, mi, counts, V, w); break;
    case 5: hipLaunchKernelGGL(k_batch_potential<5>, gm, bm, 0, s, reps, mi, counts, V, w); break;
    case 6: hipLaunchKernelGGL(k_batch_potential<6>, gm, bm, 0, s, reps, mi, counts, V, w); break;
    case 7: hipLaunchKernelGGL(k_batch_potential<7>, gm, bm, 0, s, reps, mi, counts, V, w); break;
    case 8: hipLaunchKernelGGL(k_batch_potential<8>, gm, bm, 0, s, reps, mi, counts, V, w); break;
    default: return HPF_EINVAL;
    }
    return HPF_OK;
}

static hpf_status_t batch_fields(hpf_batch* b, bool report, hipStream_t s)
{
    const BatchLayout& L = b->L;
    const int K = b->cfg.K, B = b->cfg.brick, h = b->cfg.halo;
    const int P = B + 1 + 2 * h;
    const RepK* reps = b->at<RepK>(L.off_reps);
    auto* counts = reinterpret_cast<unsigned long long*>(b->buf.counts);
    uint32_t* strays = b->at<uint32_t>(L.off_strays);
    auto* partials = b->at<unsigned long long>(L.off_partials);
    const uint32_t* cs = b->at<uint32_t>(L.off_start);
    const auto* R = reinterpret_cast<const float3*>(b->buf.R[b->rcur]);
    const uint8_t* T = b->buf.T[b->scur];
    double* w = report ? b->at<double>(L.off_wpart) : nullptr;
    if (b->pending) {
        // the last fused pass deposited the current positions: its boxes are added to the
        // counts inside the potential pass
        const dim3 gb((unsigned)b->n_brick_items), bb(kFPThreads);
        const ItemK* bi = b->at<ItemK>(L.off_brick_items);
        float* V = b->buf.V;
        switch (K) {
        case 1: hipLaunchKernelGGL(k_batch_finish_potential<1>, gb, bb, 0, s, reps, bi, B, h, partials, counts, V, w); break;
        case 2: hipLaunchKernelGGL(k_batch_finish_potential<2>, gb, bb, 0, s, reps, bi, B, h, partials, counts, V, w); break;
        case 3: hipLaunchKernelGGL(k_batch_finish_potential<3>, gb, bb, 0, s, reps, bi, B, h, partials, counts, V, w); break;
        case 4: hipLaunchKernelGGL(k_batch_finish_potential<4>, gb, bb, 0, s, reps, bi, B, h, partials, counts, V, w); break;
        case 5: hipLaunchKernelGGL(k_batch_finish_potential<5>, gb, bb, 0, s, reps, bi, B, h, partials, counts, V, w); break;
        case 6: hipLaunchKernelGGL(k_batch_finish_potential<6>, gb, bb, 0, s, reps, bi, B, h, partials, counts, V, w); break;
        case 7: hipLaunchKernelGGL(k_batch_finish_potential<7>, gb, bb, 0, s, reps, bi, B, h, partials, counts, V, w); break;
        case 8: hipLaunchKernelGGL(k_batch_finish_potential<8>, gb, bb, 0, s, reps, bi, B, h, partials, counts, V, w); break;
        default: return HPF_EINVAL;
        }
        b->pending = false;
        b->w_bricks = true;
    } else {
        const size_t smem = scatter_cells_smem(K, P);
        if (smem > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch_scatter_bricks),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess)
            return HPF_EINVAL;
        hipLaunchKernelGGL(k_zero_u32_one, dim3(1), dim3(1), 0, s, strays);
        hipLaunchKernelGGL(k_batch_scatter_bricks, dim3((unsigned)b->n_brick_items), dim3(kTcThreads), smem, s, reps,
                           b->at<ItemK>(L.off_brick_items), B, h, K, R, T, cs, partials, strays);
        hipLaunchKernelGGL(k_batch_scatter_sum<false>, dim3((unsigned)b->n_brick_items), sum_block(b->n_brick_items),
                           0, s, reps, b->at<ItemK>(L.off_brick_items), B, h, K, partials, counts);
        hipLaunchKernelGGL(k_batch_scatter_strays, dim3(256), dim3(kTcThreads), 0, s, reps, b->nrep, K, R, T, cs,
                           strays, counts);
        if (hpf_status_t st = batch_potential(b, K, counts, w, s))
            return st;
        b->w_bricks = false;
    }
    hipLaunchKernelGGL(k_batch_gradient, dim3((unsigned)b->n_planes), dim3(256), 0, s, reps,
                       b->at<ItemK>(L.off_plane_items), K, b->buf.V, reinterpret_cast<float3*>(b->buf.G));
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

using BatchAdvFn = void (*)(const RepK*, const ItemK*, int, int, int, const float3*, float3*, float3*,
                            const uint8_t*, int64_t, const float3*, const int32_t*, int, float, float, float,
                            const uint32_t*, unsigned long long*, unsigned long long*, double*, double*, int, ThermoK);

template <bool kPipe, bool kNT>
static BatchAdvFn batch_advance_fn(bool thermo, bool r0z)
{
    return thermo ? (r0z ? k_batch_advance_scatter<true, kPipe, true, kNT>
                         : k_batch_advance_scatter<false, kPipe, true, kNT>)
                  : (r0z ? k_batch_advance_scatter<true, kPipe, false, kNT>
                         : k_batch_advance_scatter<false, kPipe, false, kNT>);
}

static hpf_status_t batch_particles(hpf_batch* b, bool prime, bool report, hipStream_t s)
{
    const BatchLayout& L = b->L;
    const hpf_batch_config_t& c = b->cfg;
    const dim3 g((unsigned)b->n_bead_items), bl(kPThreads);
    const RepK* reps = b->at<RepK>(L.off_reps);
    const ItemK* items = b->at<ItemK>(L.off_bead_items);
    const auto* R = reinterpret_cast<const float3*>(b->buf.R[b->rcur]);
    auto* Rn = reinterpret_cast<float3*>(b->buf.R[1 - b->rcur]);
    auto* Vel = reinterpret_cast<float3*>(b->buf.Vel[b->scur]);
    const uint8_t* T = b->buf.T[b->scur];
    const int32_t* bonds = c.D > 0 ? b->buf.bonds[b->scur] : nullptr;
    const auto* G = reinterpret_cast<const float3*>(b->buf.G);
    double* e = report ? b->at<double>(L.off_epart) : nullptr;
    double* kp = report ? b->at<double>(L.off_kpart) : nullptr;
    const int nslot = (int)L.nslot;
    const bool fused = !prime && c.fuse_deposit;
    // the thermostat acts in every step after the start (time levels 1, 2, ... on the device)
    ThermoK th{0u, 0.0f, 0u, 0u, nullptr, nullptr, 0u};
    int64_t* tstep = b->at<int64_t>(L.off_tstep);
    if (!prime && c.thermo_p > 0.0f) {
        th.thr = c.thermo_p >= 1.0f ? (1u << 24) : (uint32_t)std::floor((double)c.thermo_p * 16777216.0);
        th.key0 = (uint32_t)c.thermo_seed;
        th.key1 = (uint32_t)(c.thermo_seed >> 32);
        th.step = tstep;
        th.tag = b->buf.tag[b->scur];
    }
    b->pending = false;
    if (fused) {
        const int P = c.brick + 1 + 2 * c.halo;
        const size_t smem = sizeof(unsigned long long) * (size_t)c.K * P * P * P;
        // the software-pipelined bead loop serves bond tables of up to kPreBonds rows and
        // gradient meshes (all replicas) of up to kBufMeshBytes
        const bool pipe = c.D <= kPreBonds && L.nm_tot * c.K * 12 <= kBufMeshBytes;
        const bool thermo = th.thr != 0, r0z = c.r0 == 0.0f;
        const int64_t bytes = L.Ntot * (49 + 4 * (int64_t)std::min(c.D, kPreBonds)) + L.nm_tot * c.K * 12 +
                              (int64_t)smem * L.bricks_tot;
        const bool nt = pipe && bytes > kStreamHintBytes;
        const BatchAdvFn fn = pipe ? (nt ? batch_advance_fn<true, true>(thermo, r0z)
                                    : batch_advance_fn<true, false>(thermo, r0z))
                              : batch_advance_fn<false, false>(thermo, r0z);
        if (smem > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess)
            return HPF_EINVAL;
        const dim3 ga((unsigned)b->n_adv_items), ba(kASThreadsBatch);
        const ItemK* adv = b->at<ItemK>(L.off_adv_items);
        const uint32_t* cs = b->at<uint32_t>(L.off_start);
        auto* partials = b->at<unsigned long long>(L.off_partials);
        auto* counts = reinterpret_cast<unsigned long long*>(b->buf.counts);
        hipLaunchKernelGGL(fn, ga, ba, smem, s, reps, adv, c.brick, c.halo, c.K, R, Rn, Vel, T, L.Ntot, G, bonds,
                           c.D, c.k_bond, c.r0, c.dt, cs, partials, counts, e, kp, nslot, th);
        b->pending = true;
    } else if (b->n_bead_items > 0) {
        if (prime) {
            if (c.r0 == 0.0f)
                hipLaunchKernelGGL(k_batch_prime<true>, g, bl, 0, s, reps, items, c.K, R, Rn, Vel, T, L.Ntot, G,
                                   bonds, c.D, c.k_bond, c.r0, c.dt, e, kp, nslot);
            else
                hipLaunchKernelGGL(k_batch_prime<false>, g, bl, 0, s, reps, items, c.K, R, Rn, Vel, T, L.Ntot, G,
                                   bonds, c.D, c.k_bond, c.r0, c.dt, e, kp, nslot);
        } else {
            using BAdvFn = void (*)(const RepK*, const ItemK*, int, const float3*, float3*, float3*, const uint8_t*,
                                    int64_t, const float3*, const int32_t*, int, float, float, float, double*,
                                    double*, int, ThermoK);
            const BAdvFn fa = th.thr ? (c.r0 == 0.0f ? k_batch_advance<true, true> : k_batch_advance<false, true>)
                                     : (c.r0 == 0.0f ? k_batch_advance<true, false> : k_batch_advance<false, false>);
            hipLaunchKernelGGL(fa, g, bl, 0, s, reps, items, c.K, R, Rn, Vel, T, L.Ntot, G, bonds, c.D, c.k_bond,
                               c.r0, c.dt, e, kp, nslot, th);
        }
    }
    if (prime)
        hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, tstep, (int64_t)1);
    else if (th.thr)
        hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(1), 0, s, tstep, (int64_t)1);
    b->rcur = 1 - b->rcur;
    if (report)
        hipLaunchKernelGGL(k_batch_reduce, dim3(b->nrep), dim3(64), 0, s,
                           b->at<int64_t>(fused ? L.off_adv_ioff : L.off_bead_ioff),
                           b->at<int64_t>(b->w_bricks ? L.off_brick_ioff : L.off_mesh_ioff),
                           b->at<double>(L.off_wpart), e, kp, nslot, b->at<double>(L.off_energy));
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

}  // namespace hpf

using namespace hpf;

extern "C" {

size_t hpf_batch_workspace_bytes(const hpf_replica_t* reps, int32_t n_rep, const hpf_batch_config_t* cfg)
{
    BatchLayout L;
    return batch_layout(reps, n_rep, cfg, &L) ? L.total : 0;
}

hpf_status_t hpf_batch_create(const hpf_replica_t* reps, int32_t n_rep, const hpf_batch_config_t* cfg,
                              const hpf_batch_buffers_t* bufs, void* work, size_t work_bytes, hpf_batch_t** out)
{
    if (!out || !bufs)
        return HPF_EINVAL;
    *out = nullptr;
    BatchLayout L;
    if (!batch_layout(reps, n_rep, cfg, &L))
        return HPF_EINVAL;
    if (!work || work_bytes < L.total)
        return HPF_ESPACE;
    hpf_batch_config_t c = *cfg;
    if (c.brick == 0)
        c.brick = 8;
    if (c.halo < 0 || c.halo > kTcMaxHalo || c.halo >= c.brick || !(c.dt > 0.0f) || c.sort_every < 0 ||
        c.bead_chunk < kMinBeadChunk || c.mesh_chunk < kMinMeshChunk || c.fuse_deposit < 0 || c.fuse_deposit > 1 ||
        !(c.thermo_p >= 0.0f && c.thermo_p <= 1.0f))
        return HPF_EINVAL;
    if (c.thermo_p > 0.0f)
        for (int r = 0; r < n_rep; ++r)
            if (!(reps[r].kT > 0.0) || !std::isfinite(reps[r].kT))
                return HPF_EINVAL;
    for (int i = 0; i < 2; ++i)
        if (L.Ntot > 0 && (!bufs->R[i] || !bufs->Vel[i] || !bufs->T[i] || !bufs->tag[i] ||
                           (c.D > 0 && !bufs->bonds[i])))
            return HPF_EINVAL;
    if (!bufs->counts || !bufs->V || !bufs->G)
        return HPF_EINVAL;
    // every bond partner must lie in its own replica: a partner in another replica would
    // couple two systems and take the wrong box's minimum image
    if (c.D > 0 && L.Ntot > 0) {
        std::vector<int32_t> tab((size_t)c.D * (size_t)L.Ntot);
        if (hipMemcpy(tab.data(), bufs->bonds[0], sizeof(int32_t) * tab.size(), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return HPF_EHIP;
        for (int r = 0; r < n_rep; ++r) {
            const int64_t lo = reps[r].bead_offset, hi = lo + reps[r].n_beads;
            for (int d = 0; d < c.D; ++d) {
                const int32_t* row = tab.data() + (size_t)d * (size_t)L.Ntot;
                for (int64_t i = lo; i < hi; ++i)
                    if (row[i] != -1 && (row[i] < lo || row[i] >= hi))
                        return HPF_EINVAL;
            }
        }
    }
    hpf_batch* b = new (std::nothrow) hpf_batch;
    if (!b)
        return HPF_EINVAL;
    b->nrep = n_rep;
    b->cfg = c;
    b->L = L;
    b->work = static_cast<char*>(work);
    b->buf = *bufs;
    b->desc.assign(reps, reps + n_rep);
    uint32_t key_base = 0;
    int64_t moff = 0, brick_off = 0;
    const int B = c.brick;
    for (int r = 0; r < n_rep; ++r) {
        const hpf_replica_t& q = reps[r];
        hpf_mesh_t mesh;
        const float Lr[3] = {q.L[0], q.L[1], q.L[2]};
        if (hpf_mesh_make(Lr, q.M, q.n_beads, &mesh) != HPF_OK) {
            delete b;
            return HPF_EINVAL;
        }
        RepK rk{};
        rk.m = mesh_k(&mesh);
        for (int d = 0; d < 3; ++d) {
            rk.box.L[d] = q.L[d];
            rk.box.halfL[d] = 0.5f * q.L[d];
            rk.nb[d] = (q.M[d] + B - 1) / B;
        }
        for (int a = 0; a < c.K; ++a)
            for (int bb = 0; bb < c.K; ++bb)
                rk.p.A[a * c.K + bb] = q.kT * q.chi[a * c.K + bb];
        rk.p.inv_kappa = q.inv_kappa;
        rk.p.rho0_dV = mesh.c_norm > 0.0 ? 1.0 / (mesh.c_norm * 281474976710656.0) : 0.0;
        rk.bead_off = q.bead_offset;
        rk.N = q.n_beads;
        rk.moff = moff;
        rk.key_base = key_base;
        rk.nbricks = (int64_t)rk.nb[0] * rk.nb[1] * rk.nb[2];
        rk.NK = (uint32_t)rk.nbricks;
        rk.brick_off = brick_off;
        rk.kT = (float)q.kT;
        key_base += rk.NK + 1;
        moff += rk.m.nm;
        brick_off += rk.nbricks;
        b->reps.push_back(rk);
    }
    if (hipMemcpy(b->work + L.off_reps, b->reps.data(), sizeof(RepK) * n_rep, hipMemcpyHostToDevice) != hipSuccess) {
        delete b;
        return HPF_EHIP;
    }
    const hpf_status_t st = batch_build_items(b);
    if (st != HPF_OK) {
        delete b;
        return st;
    }
    *out = b;
    return HPF_OK;
}

hpf_status_t hpf_batch_destroy(hpf_batch_t* b)
{
    delete b;
    return HPF_OK;
}

hpf_status_t hpf_batch_start(hpf_batch_t* b, void* stream)
{
    if (!b)
        return HPF_EINVAL;
    hipStream_t s = as_stream(stream);
    hpf_status_t st = batch_sort(b, s);
    if (st == HPF_OK)
        st = batch_fields(b, true, s);
    if (st == HPF_OK)
        st = batch_particles(b, true, true, s);
    b->steps_done = 0;
    return st;
}

hpf_status_t hpf_batch_step(hpf_batch_t* b, int32_t n_steps, int32_t report_last, void* stream)
{
    if (!b || n_steps < 0)
        return HPF_EINVAL;
    hipStream_t s = as_stream(stream);
    for (int i = 0; i < n_steps; ++i) {
        const bool report = report_last && i == n_steps - 1;
        hpf_status_t st = HPF_OK;
        if (b->cfg.sort_every > 0 && b->steps_done % b->cfg.sort_every == 0)
            st = batch_sort(b, s);
        if (st == HPF_OK)
            st = batch_fields(b, report, s);
        if (st == HPF_OK)
            st = batch_particles(b, false, report, s);
        if (st != HPF_OK)
            return st;
        ++b->steps_done;
    }
    return HPF_OK;
}

hpf_status_t hpf_batch_density(hpf_batch_t* b, uint64_t* counts_out, void* stream)
{
    if (!b || !counts_out || counts_out == b->buf.counts)
        return HPF_EINVAL;
    hipStream_t s = as_stream(stream);
    const BatchLayout& L = b->L;
    const int K = b->cfg.K, B = b->cfg.brick, h = b->cfg.halo;
    const int P = B + 1 + 2 * h;
    const RepK* reps = b->at<RepK>(L.off_reps);
    const ItemK* bi = b->at<ItemK>(L.off_brick_items);
    auto* out = reinterpret_cast<unsigned long long*>(counts_out);
    auto* partials = b->at<unsigned long long>(L.off_partials);
    if (b->n_brick_items == 0)
        return HPF_OK;
    if (b->pending) {
        // the last fused pass deposited the current positions: its strays are in the
        // batch's counts and its boxes in the partial buffer; neither is changed here
        if (hipMemcpyAsync(out, b->buf.counts, sizeof(uint64_t) * (size_t)K * (size_t)L.nm_tot,
                           hipMemcpyDeviceToDevice, s) != hipSuccess)
            return HPF_EHIP;
        hipLaunchKernelGGL(k_batch_scatter_sum<true>, dim3((unsigned)b->n_brick_items), sum_block(b->n_brick_items),
                           0, s, reps, bi, B, h, K, partials, out);
    } else {
        const size_t smem = scatter_cells_smem(K, P);
        if (smem > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch_scatter_bricks),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess)
            return HPF_EINVAL;
        uint32_t* strays = b->at<uint32_t>(L.off_strays);
        const auto* R = reinterpret_cast<const float3*>(b->buf.R[b->rcur]);
        const uint8_t* T = b->buf.T[b->scur];
        const uint32_t* cs = b->at<uint32_t>(L.off_start);
        hipLaunchKernelGGL(k_zero_u32_one, dim3(1), dim3(1), 0, s, strays);
        hipLaunchKernelGGL(k_batch_scatter_bricks, dim3((unsigned)b->n_brick_items), dim3(kTcThreads), smem, s, reps,
                           bi, B, h, K, R, T, cs, partials, strays);
        hipLaunchKernelGGL(k_batch_scatter_sum<false>, dim3((unsigned)b->n_brick_items), sum_block(b->n_brick_items),
                           0, s, reps, bi, B, h, K, partials, out);
        hipLaunchKernelGGL(k_batch_scatter_strays, dim3(256), dim3(kTcThreads), 0, s, reps, b->nrep, K, R, T, cs,
                           strays, out);
    }
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t hpf_batch_current(const hpf_batch_t* b, float** R, float** Vel, uint8_t** T, int32_t** tag,
                               int32_t** bonds, double** energies)
{
    if (!b)
        return HPF_EINVAL;
    if (R)
        *R = b->buf.R[b->rcur];
    if (Vel)
        *Vel = b->buf.Vel[b->scur];
    if (T)
        *T = b->buf.T[b->scur];
    if (tag)
        *tag = b->buf.tag[b->scur];
    if (bonds)
        *bonds = b->buf.bonds[b->scur];
    if (energies)
        *energies = reinterpret_cast<double*>(b->work + b->L.off_energy);
    return HPF_OK;
}

// Cache of tuned launch shapes by replica set (sizes, meshes, K, D) and device.
static std::mutex g_tune_mu;
static std::map<std::vector<int64_t>, hpf_batch_config_t> g_tune_cache;

static std::vector<int64_t> tune_key(const hpf_batch* b)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::vector<int64_t> k = {dev, b->nrep, b->cfg.K, b->cfg.D, b->cfg.brick, (int64_t)b->cfg.fuse_deposit};
    for (const hpf_replica_t& q : b->desc) {
        k.push_back(q.n_beads);
        for (int d = 0; d < 3; ++d)
            k.push_back(q.M[d]);
    }
    return k;
}

hpf_status_t hpf_batch_tune(hpf_batch_t* b, int32_t trial_steps, void* stream, hpf_batch_config_t* chosen,
                            float* trial_ms, int32_t* n_trials)
{
    if (!b || trial_steps < 1)
        return HPF_EINVAL;
    hipStream_t s = as_stream(stream);
    if (n_trials)
        *n_trials = 0;
    const std::vector<int64_t> key = tune_key(b);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        const auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            hpf_batch_config_t c = b->cfg;
            c.halo = it->second.halo;
            c.sort_every = it->second.sort_every;
            c.bead_chunk = it->second.bead_chunk;
            c.mesh_chunk = it->second.mesh_chunk;
            c.fuse_deposit = it->second.fuse_deposit;
            b->cfg = c;
            const hpf_status_t st = batch_build_items(b);
            if (chosen)
                *chosen = b->cfg;
            return st;
        }
    }
    // Each candidate runs from a fresh sort for a whole number of its sort intervals (trial
    // steps, at least 20, rounded up to a multiple of the interval), three times; its time
    // is the median.
    constexpr int kRepeats = 3;
    std::vector<hpf_batch_config_t> cands;
    for (int hb : {1, 2}) {
        if (hb >= b->cfg.brick)
            continue;
        for (int se : {5, 10, 20, 30, 40}) {
            hpf_batch_config_t c = b->cfg;
            c.halo = hb;
            c.sort_every = se;
            c.mesh_chunk = 16384;
            c.fuse_deposit = 1;
            cands.push_back(c);
        }
        for (int bc : {2048, 4096}) {
            hpf_batch_config_t c = b->cfg;
            c.halo = hb;
            c.sort_every = 10;
            c.mesh_chunk = 16384;
            c.fuse_deposit = 0;
            c.bead_chunk = bc;
            cands.push_back(c);
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return HPF_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return HPF_EHIP;
    }
    hpf_batch_config_t best = b->cfg;
    float best_ms = 1e30f;
    int t = 0;
    hpf_status_t st = HPF_OK;
    for (const hpf_batch_config_t& c : cands) {
        b->cfg = c;
        if ((st = batch_build_items(b)) != HPF_OK)
            break;
        const int every = c.sort_every > 0 ? c.sort_every : 1;
        const int steps = (std::max(trial_steps, 20) + every - 1) / every * every;
        float rep[kRepeats];
        for (int r = 0; r < kRepeats && st == HPF_OK; ++r) {
            b->steps_done = 0;                         // the trial starts with a sort
            if (hipEventRecord(e0, s) != hipSuccess) {
                st = HPF_EHIP;
                break;
            }
            if ((st = hpf_batch_step(b, steps, 0, stream)) != HPF_OK)
                break;
            float ms = 0.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = HPF_EHIP;
                break;
            }
            rep[r] = ms / steps;
        }
        if (st != HPF_OK)
            break;
        std::sort(rep, rep + kRepeats);
        const float med = rep[kRepeats / 2];
        if (trial_ms && t < 32)
            trial_ms[t] = med;
        ++t;
        if (med < best_ms) {
            best_ms = med;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->cfg = best;
    b->steps_done = 0;
    if (st == HPF_OK)
        st = batch_build_items(b);
    if (st == HPF_OK) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = b->cfg;
    }
    if (chosen)
        *chosen = b->cfg;
    if (n_trials)
        *n_trials = t;
    return st;
}

// ------------------------------------------------------------------ graphs

struct hpf_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

hpf_status_t hpf_graph_begin(void* stream)
{
    if (!stream)
        return HPF_EINVAL;   // the null stream cannot be captured
    return hipStreamBeginCapture(as_stream(stream), hipStreamCaptureModeThreadLocal) == hipSuccess ? HPF_OK
                                                                                                  : HPF_EHIP;
}

hpf_status_t hpf_graph_end(void* stream, hpf_graph_t** out)
{
    if (!stream || !out)
        return HPF_EINVAL;
    *out = nullptr;
    hpf_graph* g = new (std::nothrow) hpf_graph;
    if (!g)
        return HPF_EINVAL;
    if (hipStreamEndCapture(as_stream(stream), &g->graph) != hipSuccess ||
        hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        if (g->graph)
            (void)hipGraphDestroy(g->graph);
        delete g;
        return HPF_EHIP;
    }
    *out = g;
    return HPF_OK;
}

hpf_status_t hpf_graph_launch(hpf_graph_t* g, void* stream)
{
    if (!g)
        return HPF_EINVAL;
    return hipGraphLaunch(g->exec, as_stream(stream)) == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t hpf_graph_destroy(hpf_graph_t* g)
{
    if (!g)
        return HPF_EINVAL;
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    delete g;
    return HPF_OK;
}

}  // extern "C"
