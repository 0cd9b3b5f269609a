// Density assignment over the cell list (beads in hpf_sort_by_cell order).
//
// The paper gathers: one thread per mesh point collects the fractions of the
// beads in the eight cells around it (Algorithm 1 Kernel 2), so no two threads
// write one point. Here the deposit is pushed from the beads, but still
// without global atomics and with exact integer sums:
//
//   pass 1  one workgroup per B^3 brick of cells reads the beads listed in
//           the brick (a contiguous range after the sort) and accumulates
//           their fixed-point weights in an LDS box of P = B + 1 + 2h mesh
//           points per axis, h = drift halo in cells; the box is stored to a
//           per-brick partial buffer;
//   pass 2  one thread per mesh point adds the partial boxes covering it
//           (per axis the own brick and at most one neighbour) and stores the
//           count;
//   fixup   beads that moved more than h cells out of their brick since the
//           sort, and beads the sort could not bin, are added with global u64
//           atomics.
//
// Every bead is deposited exactly once, integer addition is exact and order
// free, so the counts equal those of hpf_density_scatter bit for bit.
#include "hpf_common.hpp"

namespace hpf {

constexpr int kTcThreads = 256;
constexpr int kTcMaxB = 16;
constexpr int kTcMaxHalo = 2;
constexpr int kStrayStage = 1024;   // strays a workgroup stages in LDS before appending

struct TileK {
    MeshK m;
    int32_t B;          // brick edge (tile of owned mesh points)
    int32_t h;          // drift halo in cells
    int32_t nb[3];      // bricks per axis
    uint32_t NK;        // number of sort keys (bricks); key NK = beads that cannot be binned
    int32_t P;          // B + 1 + 2h: mesh points per axis of a brick's deposit box
    int64_t ntiles;
};

// Sort key of a cell: the index of its brick of B^3 cells, x fastest.
__device__ __forceinline__ uint32_t brick_of(int cx, int cy, int cz, int B, const int nb[3])
{
    return ((uint32_t)(cz / B) * (uint32_t)nb[1] + (uint32_t)(cy / B)) * (uint32_t)nb[0] + (uint32_t)(cx / B);
}

__device__ __forceinline__ int wrap_idx(int c, int M)
{
    c %= M;
    return c < 0 ? c + M : c;
}

// Periodic difference a - b folded into [-M/2, M/2].
__device__ __forceinline__ int periodic_delta(int a, int b, int M)
{
    int d = a - b;
    if (d > M / 2)
        d -= M;
    else if (d < -(M / 2))
        d += M;
    return d;
}

__device__ __forceinline__ void lds_add_u64(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}


// Cell of bead b relative to the deposit box of the brick whose first cell is
// (x0, y0, z0) and whose width is (ox, oy, oz) cells: true, with the local
// cell (lx, ly, lz), when the bead's 8 corners lie in the part of the box that
// the sum pass reads (box points [0, o + 2h] per axis).
__device__ __forceinline__ bool brick_box_cell(const BeadCell& b, const MeshK& m, int x0, int y0, int z0, int ox,
                                               int oy, int oz, int h, int& lx, int& ly, int& lz)
{
    lx = periodic_delta(b.c[0], x0, m.M[0]) + h;
    ly = periodic_delta(b.c[1], y0, m.M[1]) + h;
    lz = periodic_delta(b.c[2], z0, m.M[2]) + h;
    return lx >= 0 && lx <= ox - 1 + 2 * h && ly >= 0 && ly <= oy - 1 + 2 * h && lz >= 0 && lz <= oz - 1 + 2 * h;
}

// yz * q for yz <= 2^32 and q < 2^16, exactly: two products of at most 17 x 16 bits,
// which the 24-bit multiplier forms at full rate.
__device__ __forceinline__ uint64_t mul_w16(uint64_t yz, uint32_t q)
{
    const uint32_t yh = (uint32_t)(yz >> HPF_FIX_BITS) & 0x1ffffu, yl = (uint32_t)yz & 0xffffu;
    return ((uint64_t)(yh * q) << HPF_FIX_BITS) + (uint64_t)(yl * q);
}

// Adds one bead's 8 fixed-point corner weights to species t of an LDS box of
// P^3 points at local cell (lx, ly, lz). The corner weights come from two
// products: with w0 = 2^S - w1 per axis, W(0, ., .) = 2^S W_yz - W(1, ., .),
// and likewise along y and z. Every q is below 2^16 (cell_coord), so the masks
// change nothing; they let the compiler use the 24-bit multiplier.

__device__ __forceinline__ void box_deposit(unsigned long long* box, int P, int t, int lx, int ly, int lz,
                                            const BeadCell& b)
{
    const int P2 = P * P;
    const uint32_t q0 = b.q[0] & 0xffffu, q1 = b.q[1] & 0xffffu, q2 = b.q[2] & 0xffffu;
    const uint32_t yz11 = q1 * q2;
    const uint32_t yz01 = (q2 << HPF_FIX_BITS) - yz11;   // wy0 wz1
    const uint32_t yz10 = (q1 << HPF_FIX_BITS) - yz11;   // wy1 wz0
    const uint64_t yz00 = ((uint64_t)kOne << HPF_FIX_BITS) - yz11 - yz01 - yz10;
    unsigned long long* c0 = box + t * P2 * P + (lz * P + ly) * P + lx;
    const uint64_t a00 = mul_w16(yz00, q0), a10 = mul_w16(yz10, q0);
    const uint64_t a01 = mul_w16(yz01, q0), a11 = mul_w16(yz11, q0);
    lds_add_u64(c0, (yz00 << HPF_FIX_BITS) - a00);
    lds_add_u64(c0 + 1, a00);
    lds_add_u64(c0 + P, ((uint64_t)yz10 << HPF_FIX_BITS) - a10);
    lds_add_u64(c0 + P + 1, a10);
    lds_add_u64(c0 + P2, ((uint64_t)yz01 << HPF_FIX_BITS) - a01);
    lds_add_u64(c0 + P2 + 1, a01);
    lds_add_u64(c0 + P2 + P, ((uint64_t)yz11 << HPF_FIX_BITS) - a11);
    lds_add_u64(c0 + P2 + P + 1, a11);
}

// Pass 1: one workgroup per brick deposits the beads listed in that brick --
// one contiguous range of the cell-sorted arrays -- into an LDS box of
// P = B + 1 + 2h mesh points per axis starting h points below the brick (a
// bead that drifted at most h cells reaches points [x0 - h, x0 + B + h]). A
// thread takes kScBatch consecutive beads, so the lanes of one LDS atomic
// mostly sit in different cells. The box goes to a per-brick partial buffer
// with plain stores. Beads outside the box (strays) and beads that cannot be
// binned are staged and appended to the stray list.
constexpr int kScBatch = 4;

// Deposit of the beads listed in `brick` (cell_start of this system, i.e.
// already offset for batched systems) into an LDS box, stored to `out`.
__device__ __forceinline__ void scatter_brick_body(const float3* __restrict__ R, const uint8_t* __restrict__ T,
                                                   int K, const TileK& tk,
                                                   const uint32_t* __restrict__ cell_start, int64_t brick,
                                                   unsigned long long* __restrict__ out,
                                                   uint32_t* __restrict__ strays)
{
    extern __shared__ unsigned long long smem[];
    __shared__ uint32_t stray_buf[kStrayStage];
    __shared__ uint32_t stray_n, stray_base;
    const int tid = threadIdx.x;
    const int B = tk.B, h = tk.h, P = tk.P;
    const int Mx = tk.m.M[0], My = tk.m.M[1], Mz = tk.m.M[2];
    const int bx = (int)(brick % tk.nb[0]);
    const int by = (int)((brick / tk.nb[0]) % tk.nb[1]);
    const int bz = (int)(brick / ((int64_t)tk.nb[0] * tk.nb[1]));
    const int x0 = bx * B, y0 = by * B, z0 = bz * B;
    const int ox = min(B, Mx - x0), oy = min(B, My - y0), oz = min(B, Mz - z0);
    const int P2 = P * P, P3 = P2 * P;
    const int nbox = K * P3;
    unsigned long long* box = smem;
    for (int e = tid; e < nbox; e += kTcThreads)
        box[e] = 0ull;
    if (tid == 0)
        stray_n = 0;
    __syncthreads();
    const uint32_t first = cell_start[brick];
    const uint32_t last = cell_start[brick + 1];
    for (uint32_t j0 = first; j0 < last; j0 += kTcThreads * kScBatch) {
        float3 rj[kScBatch];
        int tj[kScBatch];
        const uint32_t jb = j0 + tid * kScBatch;
#pragma unroll
        for (int u = 0; u < kScBatch; ++u) {
            if (jb + u < last) {
                rj[u] = R[jb + u];
                tj[u] = T[jb + u];
            }
        }
#pragma unroll
        for (int u = 0; u < kScBatch; ++u) {
            const uint32_t p = jb + u;
            if (p >= last)
                continue;
            const int t = tj[u];
            BeadCell b;
            int lx, ly, lz;
            const bool ok = bead_cell(rj[u], tk.m, b) && t < K;
            if (!ok || !brick_box_cell(b, tk.m, x0, y0, z0, ox, oy, oz, h, lx, ly, lz)) {
                const uint32_t slot = atomicAdd(&stray_n, 1u);
                if (slot < (uint32_t)kStrayStage)
                    stray_buf[slot] = p;
                else
                    strays[1 + atomicAdd(strays, 1u)] = p;       // stage full: direct append
                continue;
            }
            box_deposit(box, P, t, lx, ly, lz, b);
        }
    }
    __syncthreads();
    // one global reservation per workgroup for its staged strays
    const uint32_t nst = min(stray_n, (uint32_t)kStrayStage);
    if (tid == 0 && nst)
        stray_base = atomicAdd(strays, nst);
    __syncthreads();
    for (uint32_t i = tid; i < nst; i += kTcThreads)
        strays[1 + stray_base + i] = stray_buf[i];
    for (int e = tid; e < nbox; e += kTcThreads)
        out[e] = box[e];
}

__global__ __launch_bounds__(kTcThreads) void k_scatter_bricks(const float3* __restrict__ R,
                                                               const uint8_t* __restrict__ T, int K,
                                                               TileK tk,
                                                               const uint32_t* __restrict__ cell_start,
                                                               unsigned long long* __restrict__ partials,
                                                               uint32_t* __restrict__ strays)
{
    const int64_t brick = xcd_block(blockIdx.x, gridDim.x);
    const int P = tk.P;
    scatter_brick_body(R, T, K, tk, cell_start, brick, partials + brick * (int64_t)K * P * P * P, strays);
}

// Pass 2: one thread per mesh point sums the partial boxes that cover it and
// stores the count. Along an axis the box of brick b spans points
// [bB - h, bB + ob + h] (ob = the brick's width), periodically. With h < B
// only bricks b0 - 2 .. b0 + 2 (b0 = v / B) can reach v; the +-2 ones matter
// only next to the periodic seam when the last brick is narrower than h.
struct Cover {
    int n;
    int64_t off[5];     // brick * (brick stride) + local * (point stride) along this axis
};

// Writes into c (in LDS) the boxes that cover coordinate v along one axis. A
// brick reached twice through the periodic wrap (fewer than five bricks on the
// axis) is listed once. Brick numbers are kept in registers (constant indices
// only), so nothing of this goes to scratch memory.
__device__ __forceinline__ void covering(Cover& c, int v, int B, int h, int nb, int M, int64_t bstride,
                                         int lstride)
{
    int n = 0;
    int seen[5];
    const int b0 = v / B;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        int b = b0 + q - 2;
        if (b < 0)
            b += nb;
        else if (b >= nb)
            b -= nb;
        bool ok = b >= 0 && b < nb;         // fewer than 3 bricks on this axis
        seen[q] = ok ? b : -1 - q;
#pragma unroll
        for (int r = 0; r < q; ++r)
            ok &= seen[r] != b;
        const int ob = min(B, M - b * B);
        int l = v - (b * B - h);
        if (l < 0)
            l += M;
        else if (l >= M)
            l -= M;
        if (ok && l <= ob + 2 * h) {
            c.off[n] = b * bstride + (int64_t)l * lstride;
            ++n;
        }
    }
    c.n = n;
}

// The entries that cover one point when no axis has more than two covering
// boxes (the usual case): the eight offsets and which of them exist. Built and
// read with constant indices only, so it stays in registers.
struct Cover2 {
    int64_t e[8];
    bool use[8];
};

__device__ __forceinline__ bool cover2_ok(const Cover& cx, const Cover& cy, const Cover& cz)
{
    return cx.n <= 2 && cy.n <= 2 && cz.n <= 2;
}

__device__ __forceinline__ Cover2 cover2(const Cover& cx, const Cover& cy, const Cover& cz)
{
    const bool hx = cx.n > 1, hy = cy.n > 1, hz = cz.n > 1;
    const int64_t x[2] = {cx.off[0], hx ? cx.off[1] : cx.off[0]};
    const int64_t y[2] = {cy.off[0], hy ? cy.off[1] : cy.off[0]};
    const int64_t z[2] = {cz.off[0], hz ? cz.off[1] : cz.off[0]};
    Cover2 c;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = q >> 2, b = (q >> 1) & 1, d = q & 1;
        c.e[q] = z[a] + y[b] + x[d];
        c.use[q] = (a == 0 || hz) && (b == 0 || hy) && (d == 0 || hx);
    }
    return c;
}

// Sum of the covering entries of species block kb (= k * P^3); every load of
// the point is issued before the additions.
__device__ __forceinline__ unsigned long long cover2_sum(const unsigned long long* __restrict__ partials,
                                                         const Cover2& c, int64_t kb)
{
    unsigned long long v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        v[q] = c.use[q] ? partials[c.e[q] + kb] : 0ull;
    unsigned long long sum = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        sum += v[q];
    return sum;
}

// One of three values by axis, selected as values (the arguments are copies).
__device__ __forceinline__ int pick3(int d, int a, int b, int c) { return d == 0 ? a : d == 1 ? b : c; }

// Cover lists of one brick's coordinates along each axis, with the offsets of
// the covering boxes' entries precomputed per axis (the offset of an entry in
// the partial buffer is the sum of its three axis terms), so that a point's
// covering entries cost three additions each. Call with all threads; ends
// with a barrier.
__device__ __forceinline__ void brick_covers(Cover (&cov)[3][kTcMaxB], const TileK& tk, int K, const int bxyz[3],
                                             const int o[3])
{
    const int B = tk.B, h = tk.h, P = tk.P;
    const int64_t P3K = (int64_t)K * P * P * P;
    const int tid = threadIdx.x;
    if (tid < 3 * B) {
        // the axis is chosen among values: a run-time index into the per-axis arrays
        // (or a conditional over them, which selects an address) would place them in
        // scratch memory
        const int d = tid / B, i = tid % B;
        const int od = pick3(d, o[0], o[1], o[2]);
        if (i < od) {
            const int bd = pick3(d, bxyz[0], bxyz[1], bxyz[2]);
            const int nbd = pick3(d, tk.nb[0], tk.nb[1], tk.nb[2]);
            const int Md = pick3(d, tk.m.M[0], tk.m.M[1], tk.m.M[2]);
            const int64_t bstride = d == 0 ? P3K : d == 1 ? tk.nb[0] * P3K : (int64_t)tk.nb[0] * tk.nb[1] * P3K;
            const int lstride = pick3(d, 1, P, P * P);
            covering(cov[d][i], bd * B + i, B, h, nbd, Md, bstride, lstride);
        }
    }
    __syncthreads();
}

// Local coordinates of point e of a brick of o[0] x o[1] x o[2] points (x fastest).
__device__ __forceinline__ void brick_point(int e, const int o[3], int B, int& ix, int& iy, int& iz)
{
    if (B == 8 && o[0] == 8 && o[1] == 8) {
        ix = e & 7;
        iy = (e >> 3) & 7;
        iz = e >> 6;
    } else {
        ix = e % o[0];
        const int r1 = e / o[0];
        iy = r1 % o[1];
        iz = r1 / o[1];
    }
}

// One workgroup per brick: the cover lists of the brick's coordinates along
// each axis are built once in LDS, then each thread sums the partial boxes for
// its points (consecutive threads -> consecutive x -> coalesced reads).
// With kAdd the sums are added to the counts instead of stored.
template <bool kAdd = false>
__device__ __forceinline__ void scatter_sum_body(const unsigned long long* __restrict__ partials,
                                                 const TileK& tk, int K, int64_t brick,
                                                 unsigned long long* __restrict__ counts)
{
    __shared__ Cover cov[3][kTcMaxB];
    const int B = tk.B, P = tk.P, P3 = P * P * P;
    const int bxyz[3] = {(int)(brick % tk.nb[0]), (int)((brick / tk.nb[0]) % tk.nb[1]),
                         (int)(brick / ((int64_t)tk.nb[0] * tk.nb[1]))};
    int o[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        o[d] = min(B, tk.m.M[d] - bxyz[d] * B);
    brick_covers(cov, tk, K, bxyz, o);
    const int npts = o[0] * o[1] * o[2];
    const int Mx = tk.m.M[0], My = tk.m.M[1];
    for (int e = threadIdx.x; e < npts; e += (int)blockDim.x) {
        int ix, iy, iz;
        brick_point(e, o, B, ix, iy, iz);
        const Cover& cx = cov[0][ix];
        const Cover& cy = cov[1][iy];
        const Cover& cz = cov[2][iz];
        const int64_t dst = ((int64_t)(bxyz[2] * B + iz) * My + (bxyz[1] * B + iy)) * Mx + bxyz[0] * B + ix;
        if (cover2_ok(cx, cy, cz)) {
            const Cover2 c2 = cover2(cx, cy, cz);
            for (int k = 0; k < K; ++k) {
                const unsigned long long sum = cover2_sum(partials, c2, (int64_t)k * P3);
                if (kAdd)
                    counts[(int64_t)k * tk.m.nm + dst] += sum;
                else
                    counts[(int64_t)k * tk.m.nm + dst] = sum;
            }
            continue;
        }
        for (int k = 0; k < K; ++k) {
            unsigned long long sum = 0;
            for (int a = 0; a < cz.n; ++a)
                for (int b2 = 0; b2 < cy.n; ++b2)
                    for (int c = 0; c < cx.n; ++c)
                        sum += partials[cz.off[a] + cy.off[b2] + cx.off[c] + (int64_t)k * P3];
            if (kAdd)
                counts[(int64_t)k * tk.m.nm + dst] += sum;
            else
                counts[(int64_t)k * tk.m.nm + dst] = sum;
        }
    }
}

// Up to one thread per point of the brick (B^3 <= 512): launched with 512
// threads when there are few bricks (a small mesh must still fill the chip),
// else with 256.
constexpr int kSumThreads = 512;
constexpr int64_t kSumFewBricks = 2048;

static dim3 sum_block(int64_t ntiles) { return dim3(ntiles < kSumFewBricks ? kSumThreads : kSumThreads / 2); }

template <bool kAdd>
__global__ __launch_bounds__(kSumThreads) void k_scatter_sum(const unsigned long long* __restrict__ partials,
                                                     TileK tk, int K,
                                                     unsigned long long* __restrict__ counts)
{
    scatter_sum_body<kAdd>(partials, tk, K, xcd_block(blockIdx.x, gridDim.x), counts);
}

__device__ __forceinline__ void atomic_add_u64_agent(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Eight global u64 atomics of one bead; false if it cannot be binned.
__device__ __forceinline__ bool deposit_global(const float3& r, int t, int K, const MeshK& m,
                                               unsigned long long* __restrict__ counts)
{
    BeadCell b;
    if (!(bead_cell(r, m, b) && t < K))
        return false;
    const int32_t x0 = b.c[0], x1 = next_wrap(x0, m.M[0]);
    const int32_t y0 = b.c[1], y1 = next_wrap(y0, m.M[1]);
    const int32_t z0 = b.c[2], z1 = next_wrap(z0, m.M[2]);
    const uint64_t wx0 = kOne - b.q[0], wx1 = b.q[0];
    const uint64_t wy0 = kOne - b.q[1], wy1 = b.q[1];
    const uint64_t wz0 = kOne - b.q[2], wz1 = b.q[2];
    unsigned long long* nk = counts + (int64_t)t * m.nm;
    const int64_t r00 = ((int64_t)z0 * m.M[1] + y0) * m.M[0];
    const int64_t r10 = ((int64_t)z0 * m.M[1] + y1) * m.M[0];
    const int64_t r01 = ((int64_t)z1 * m.M[1] + y0) * m.M[0];
    const int64_t r11 = ((int64_t)z1 * m.M[1] + y1) * m.M[0];
    atomic_add_u64_agent(nk + r00 + x0, wx0 * wy0 * wz0);
    atomic_add_u64_agent(nk + r00 + x1, wx1 * wy0 * wz0);
    atomic_add_u64_agent(nk + r10 + x0, wx0 * wy1 * wz0);
    atomic_add_u64_agent(nk + r10 + x1, wx1 * wy1 * wz0);
    atomic_add_u64_agent(nk + r01 + x0, wx0 * wy0 * wz1);
    atomic_add_u64_agent(nk + r01 + x1, wx1 * wy0 * wz1);
    atomic_add_u64_agent(nk + r11 + x0, wx0 * wy1 * wz1);
    atomic_add_u64_agent(nk + r11 + x1, wx1 * wy1 * wz1);
    return true;
}

// Global-atomic deposit of the stray beads and of the beads the sort could not
// bin (storage indices [cell_start[NK], N)).
__global__ __launch_bounds__(kTcThreads) void k_scatter_strays(const float3* __restrict__ R,
                                                               const uint8_t* __restrict__ T, int64_t N,
                                                               int K, MeshK m, uint32_t NK,
                                                               const uint32_t* __restrict__ cell_start,
                                                               const uint32_t* __restrict__ strays,
                                                               unsigned long long* __restrict__ counts)
{
    const int64_t nstray = strays[0];
    const int64_t tail0 = cell_start[NK];
    const int64_t total = nstray + (N - tail0);
    bool bad = false;
    for (int64_t j = (int64_t)blockIdx.x * kTcThreads + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * kTcThreads) {
        const int64_t p = j < nstray ? (int64_t)strays[1 + j] : tail0 + (j - nstray);
        bad |= !deposit_global(R[p], T[p], K, m, counts);
    }
    if (bad)
        raise_flag(HPF_FLAG_BAD_BEAD);
}

__global__ void k_zero_u32_one(uint32_t* p) { *p = 0u; }

size_t scatter_cells_smem(int K, int P)
{
    return sizeof(unsigned long long) * (size_t)K * P * P * P;
}

size_t scatter_cells_partials(int64_t ntiles, int K, int P)
{
    return sizeof(unsigned long long) * (size_t)ntiles * K * P * P * P;
}

hpf_status_t launch_scatter_cells(const float* R, const uint8_t* T, int64_t N, const TileK& tk, int K,
                                  const uint32_t* cell_start, uint64_t* counts, uint32_t* strays,
                                  unsigned long long* partials, hipStream_t s)
{
    auto* c = reinterpret_cast<unsigned long long*>(counts);
    auto* Rp = reinterpret_cast<const float3*>(R);
    const size_t smem = scatter_cells_smem(K, tk.P);
    if (smem > 65536) {
        // gfx950 has 160 KiB of LDS per CU; opt in above the 64 KiB default
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(k_scatter_bricks),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess)
            return HPF_EINVAL;
    }
    hipLaunchKernelGGL(k_zero_u32_one, dim3(1), dim3(1), 0, s, strays);
    hipLaunchKernelGGL(k_scatter_bricks, dim3((unsigned)tk.ntiles), dim3(kTcThreads), smem, s, Rp, T, K, tk,
                       cell_start, partials, strays);
    hipLaunchKernelGGL(k_scatter_sum<false>, dim3((unsigned)tk.ntiles), sum_block(tk.ntiles), 0, s, partials, tk, K,
                       c);
    hipLaunchKernelGGL(k_scatter_strays, dim3(512), dim3(kTcThreads), 0, s, Rp, T, N, K, tk.m, tk.NK,
                       cell_start, strays, c);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

}  // namespace hpf
