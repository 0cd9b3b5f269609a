// Canonical cell ordering of the beads (the paper reorders particle data for
// cache hits and bins beads into a cell list, Algorithm 1 Kernel 1).
//
// The key of a bead is the brick of B^3 cells holding its cell. Counting sort
// on that key: histogram (u32 atomics), an exclusive scan over all keys,
// placement with per-key cursors, then each key's segment is sorted by tag in
// LDS, so the result -- ascending (brick, tag) -- is independent of the
// atomic placement order. Inside a brick the beads then lie in tag order, so
// the beads of one chain (consecutive tags) stay next to each other and most
// bond partners are neighbours in memory. Finally the bead arrays are
// gathered into the output buffers and the bond table is permuted and
// renumbered through the inverse permutation.
#include "hpf_common.hpp"

namespace hpf {

struct SortK {
    MeshK m;
    int32_t B;
    int32_t nb[3];
    uint32_t NK;        // number of keys (bricks); key NK = "cannot be binned"
};

constexpr int kSortThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kSortThreads * kScanPer;   // entries per scan block
constexpr int kScanTopThreads = 1024;
constexpr int kScanTopPer = 8;
constexpr int kMaxScanTiles = kScanTopThreads * kScanTopPer;
constexpr int kBrickSortThreads = 512;
constexpr int kBrickSortMax = 8192;                    // longest segment sorted by tag (64 KB LDS)

__global__ __launch_bounds__(kSortThreads) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kSortThreads)
        p[i] = v;
}

__global__ __launch_bounds__(kSortThreads) void k_copy_u32(const uint32_t* __restrict__ a,
                                                           uint32_t* __restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kSortThreads)
        b[i] = a[i];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_keys(const float4* __restrict__ R, int64_t N,
                                                            SortK sk, uint32_t* __restrict__ keys,
                                                            uint32_t* __restrict__ hist)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * kSortThreads + threadIdx.x;
    const bool active = i < N;
    uint32_t key = sk.NK;
    if (active) {
        BeadCell b;
        if (bead_cell(R[i], sk.m, b))
            key = brick_of(b.c[0], b.c[1], b.c[2], sk.B, sk.nb);
        keys[i] = key;
    }
    // one atomic per distinct key of the wavefront
    const uint64_t grp = wave_key_group(key, active);
    const int lane = threadIdx.x & (kWave - 1);
    if (active && __builtin_ctzll(grp) == lane)
        atomicAdd(hist + key, (uint32_t)__builtin_popcountll(grp));
}

// Per-tile exclusive scan in place; tile totals to tile_sums.
__global__ __launch_bounds__(kSortThreads) void k_scan_tiles(uint32_t* __restrict__ a, int64_t n,
                                                             uint32_t* __restrict__ tile_sums)
{
    __shared__ uint32_t sh[kSortThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = base + j < n ? a[base + j] : 0u;
        sum += v[j];
    }
    uint32_t total;
    uint32_t run = block_excl_scan<kSortThreads>(sum, sh, &total);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        if (base + j < n)
            a[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0)
        tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanTopThreads) void k_scan_top(uint32_t* __restrict__ t, int n)
{
    __shared__ uint32_t sh[kScanTopThreads / kWave + 1];
    const int base = threadIdx.x * kScanTopPer;
    uint32_t v[kScanTopPer];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanTopPer; ++j) {
        v[j] = base + j < n ? t[base + j] : 0u;
        sum += v[j];
    }
    uint32_t total;
    uint32_t run = block_excl_scan<kScanTopThreads>(sum, sh, &total);
#pragma unroll
    for (int j = 0; j < kScanTopPer; ++j) {
        if (base + j < n)
            t[base + j] = run;
        run += v[j];
    }
}

__global__ __launch_bounds__(kSortThreads) void k_scan_add(uint32_t* __restrict__ a, int64_t n,
                                                           const uint32_t* __restrict__ tile_sums)
{
    const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
    if (i < n)
        a[i] += tile_sums[i / kScanTile];
}

// Placement: each group of equal keys in a wavefront reserves its slots with
// one atomic; tags travel with the permutation so the in-brick sort reads
// them contiguously.
__global__ __launch_bounds__(kSortThreads) void k_sort_place(const uint32_t* __restrict__ keys, int64_t N,
                                                             const int32_t* __restrict__ tag,
                                                             uint32_t* __restrict__ cursor,
                                                             int32_t* __restrict__ perm,
                                                             int32_t* __restrict__ ptag)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * kSortThreads + threadIdx.x;
    const bool active = i < N;
    const uint32_t key = active ? keys[i] : 0xffffffffu;
    const uint64_t grp = wave_key_group(key, active);
    const int lane = threadIdx.x & (kWave - 1);
    const int leader = active ? __builtin_ctzll(grp) : lane;
    uint32_t base = 0;
    if (active && leader == lane)
        base = atomicAdd(cursor + key, (uint32_t)__builtin_popcountll(grp));
    base = __shfl(base, leader, kWave);
    if (active) {
        const uint32_t pos = base + (uint32_t)__builtin_popcountll(grp & ((1ull << lane) - 1));
        perm[pos] = (int32_t)i;
        ptag[pos] = tag ? tag[i] : (int32_t)i;
    }
}

// Sort every key's segment of (perm, ptag) by tag (by input index when there
// are no tags): one workgroup per segment runs a bitonic sort of (tag, perm)
// pairs, padded to a power of two (at least one element per thread) with
// entries that sort last. Element e = r * 512 + t lives in register row r of
// thread t: compare-exchange partners at distance j >= 512 are in the same
// thread, at j < 64 in the same wavefront (lane shuffles), and only
// 64 <= j < 512 go through LDS. Tags compare as signed integers; they are
// unique, so perm breaks no ties. A segment longer than kBrickSortMax keeps
// its placement order and raises HPF_FLAG_SORT_ORDER.

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, kWave);
    return ((unsigned long long)hi << 32) | lo;
}

// compare-exchange of register rows r and r + D (D = j / 512) for r with bit D clear
template <int D, int ROWS>
__device__ __forceinline__ void bitonic_rows(unsigned long long (&v)[ROWS], uint32_t t, uint32_t k)
{
    if constexpr (D < ROWS) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            if ((r & D) == 0) {
                const uint32_t e = (uint32_t)r * kBrickSortThreads + t;
                const unsigned long long x = v[r], y = v[r | D];
                const bool sw = (x > y) == ((e & k) == 0);
                v[r] = sw ? y : x;
                v[r | D] = sw ? x : y;
            }
        }
    }
}

// Bitonic sort of one segment of n <= ROWS * 512 entries starting at a.
template <int ROWS>
__device__ __forceinline__ void sort_segment(uint32_t a, uint32_t n, int32_t* __restrict__ ptag,
                                             int32_t* __restrict__ perm, unsigned long long* sh)
{
    const uint32_t t = threadIdx.x;
    constexpr uint32_t np = (uint32_t)ROWS * kBrickSortThreads;
    unsigned long long v[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const uint32_t e = (uint32_t)r * kBrickSortThreads + t;
        v[r] = e < n ? ((unsigned long long)((uint32_t)ptag[a + e] ^ 0x80000000u) << 32) | (uint32_t)perm[a + e]
                     : ~0ull;
    }
    for (uint32_t k = 2; k <= np; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            if (j >= (uint32_t)kBrickSortThreads) {
                const uint32_t d = j / kBrickSortThreads;
                if (d == 1)
                    bitonic_rows<1, ROWS>(v, t, k);
                else if (d == 2)
                    bitonic_rows<2, ROWS>(v, t, k);
                else if (d == 4)
                    bitonic_rows<4, ROWS>(v, t, k);
                else
                    bitonic_rows<8, ROWS>(v, t, k);
            } else if (j >= (uint32_t)kWave) {
                __syncthreads();                       // earlier reads of sh are done
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
                    sh[r * kBrickSortThreads + t] = v[r];
                __syncthreads();
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    const uint32_t e = (uint32_t)r * kBrickSortThreads + t, p = e ^ j;
                    const unsigned long long x = v[r], y = sh[p];
                    const bool keep_min = (e < p) == ((e & k) == 0);
                    v[r] = keep_min == (x < y) ? x : y;
                }
            } else {
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    const uint32_t e = (uint32_t)r * kBrickSortThreads + t;
                    const unsigned long long x = v[r], y = shfl_xor_u64(x, (int)j);
                    const bool keep_min = (t & j) == 0 ? ((e & k) == 0) : ((e & k) != 0);
                    v[r] = keep_min == (x < y) ? x : y;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const uint32_t e = (uint32_t)r * kBrickSortThreads + t;
        if (e < n) {
            ptag[a + e] = (int32_t)((uint32_t)(v[r] >> 32) ^ 0x80000000u);
            perm[a + e] = (int32_t)(uint32_t)v[r];
        }
    }
}

__global__ __launch_bounds__(kBrickSortThreads, 4) void k_sort_bricks(const uint32_t* __restrict__ start,
                                                                   int64_t nseg, int32_t* __restrict__ ptag,
                                                                   int32_t* __restrict__ perm)
{
    __shared__ unsigned long long sh[kBrickSortMax];
    for (int64_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        const uint32_t a = start[seg], b = start[seg + 1];
        const uint32_t n = b - a;
        if (n <= 1)
            continue;
        if (n > (uint32_t)kBrickSortMax) {
            if (threadIdx.x == 0)
                raise_flag(HPF_FLAG_SORT_ORDER);
            continue;
        }
        if (n <= 512)
            sort_segment<1>(a, n, ptag, perm, sh);
        else if (n <= 1024)
            sort_segment<2>(a, n, ptag, perm, sh);
        else if (n <= 2048)
            sort_segment<4>(a, n, ptag, perm, sh);
        else if (n <= 4096)
            sort_segment<8>(a, n, ptag, perm, sh);
        else
            sort_segment<16>(a, n, ptag, perm, sh);
        __syncthreads();                               // sh is free for the next segment
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_permute(const int32_t* __restrict__ perm, int64_t N,
                                                               const float4* __restrict__ R_in,
                                                               const float4* __restrict__ V_in,
                                                               const uint8_t* __restrict__ T_in,
                                                               const int32_t* __restrict__ tag_in,
                                                               float4* __restrict__ R_out,
                                                               float4* __restrict__ V_out,
                                                               uint8_t* __restrict__ T_out,
                                                               int32_t* __restrict__ tag_out,
                                                               int32_t* __restrict__ inv)
{
    const int64_t p = xcd_block(blockIdx.x, gridDim.x) * kSortThreads + threadIdx.x;
    if (p >= N)
        return;
    const int32_t o = perm[p];
    R_out[p] = R_in[o];
    if (V_in)
        V_out[p] = V_in[o];
    T_out[p] = T_in[o];
    if (tag_in)
        tag_out[p] = tag_in[o];
    inv[o] = (int32_t)p;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_bonds(const int32_t* __restrict__ perm,
                                                             const int32_t* __restrict__ inv, int64_t N,
                                                             const int32_t* __restrict__ bonds_in, int D,
                                                             int32_t* __restrict__ bonds_out)
{
    const int64_t p = xcd_block(blockIdx.x, gridDim.x) * kSortThreads + threadIdx.x;
    if (p >= N)
        return;
    const int32_t o = perm[p];
    bool bad = false;
    for (int b = 0; b < D; ++b) {
        const int32_t j = bonds_in[(int64_t)b * N + o];
        int32_t nj = -1;
        if (j >= 0 && j < N)
            nj = inv[j];
        else if (j >= N || j < -1)
            bad = true;
        bonds_out[(int64_t)b * N + p] = nj;
    }
    if (bad)
        raise_flag(HPF_FLAG_BAD_BOND);
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool sort_layout(int64_t N, const int32_t M[3], int B, SortK* sk_out, size_t* bytes,
                 size_t off[7])
{
    if (B == 0)
        B = 8;
    if (B < 1 || B > 16 || N < 0 || N > 0x7ffffff0LL)
        return false;
    int64_t nk = 1;
    int32_t nb[3];
    for (int d = 0; d < 3; ++d) {
        nb[d] = (M[d] + B - 1) / B;
        nk *= nb[d];
    }
    const int64_t nscan = nk + 2;
    const int64_t ntiles = (nscan + kScanTile - 1) / kScanTile;
    if (ntiles > kMaxScanTiles)
        return false;
    if (sk_out) {
        sk_out->B = B;
        for (int d = 0; d < 3; ++d)
            sk_out->nb[d] = nb[d];
        sk_out->NK = (uint32_t)nk;
    }
    size_t o = 0;
    off[0] = o; o += align_up(sizeof(uint32_t) * (size_t)(N > 0 ? N : 1));    // keys
    off[1] = o; o += align_up(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));     // perm
    off[2] = o; o += align_up(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));     // inv
    off[3] = o; o += align_up(sizeof(uint32_t) * (size_t)nscan);              // start
    off[4] = o; o += align_up(sizeof(uint32_t) * (size_t)nscan);              // cursor
    off[5] = o; o += align_up(sizeof(uint32_t) * (size_t)ntiles);             // tile sums
    off[6] = o; o += align_up(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));     // tags in perm order
    *bytes = o;
    return true;
}

static unsigned grid_for(int64_t n) { return (unsigned)((n + kSortThreads - 1) / kSortThreads); }

hpf_status_t launch_sort(const SortK& sk, int64_t N, const float* R_in, const float* V_in,
                         const uint8_t* T_in, const int32_t* tag_in, const int32_t* bonds_in, int D,
                         float* R_out, float* V_out, uint8_t* T_out, int32_t* tag_out,
                         int32_t* bonds_out, uint32_t* cell_start, char* work, const size_t off[7],
                         hipStream_t s)
{
    uint32_t* keys = reinterpret_cast<uint32_t*>(work + off[0]);
    int32_t* perm = reinterpret_cast<int32_t*>(work + off[1]);
    int32_t* inv = reinterpret_cast<int32_t*>(work + off[2]);
    uint32_t* start = cell_start ? cell_start : reinterpret_cast<uint32_t*>(work + off[3]);
    uint32_t* cursor = reinterpret_cast<uint32_t*>(work + off[4]);
    uint32_t* tiles = reinterpret_cast<uint32_t*>(work + off[5]);
    int32_t* ptag = reinterpret_cast<int32_t*>(work + off[6]);
    const int64_t nscan = (int64_t)sk.NK + 2;
    const int64_t ntiles = (nscan + kScanTile - 1) / kScanTile;
    const unsigned gfill = (unsigned)std::min<int64_t>(grid_for(nscan), 4096);

    hipLaunchKernelGGL(k_fill_u32, dim3(gfill), dim3(kSortThreads), 0, s, start, nscan, 0u);
    if (N > 0)
        hipLaunchKernelGGL(k_sort_keys, dim3(grid_for(N)), dim3(kSortThreads), 0, s,
                           reinterpret_cast<const float4*>(R_in), N, sk, keys, start);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, start, nscan,
                       tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTopThreads), 0, s, tiles, (int)ntiles);
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(nscan)), dim3(kSortThreads), 0, s, start, nscan,
                       tiles);
    if (N > 0) {
        hipLaunchKernelGGL(k_copy_u32, dim3(gfill), dim3(kSortThreads), 0, s, start, cursor, nscan);
        hipLaunchKernelGGL(k_sort_place, dim3(grid_for(N)), dim3(kSortThreads), 0, s, keys, N,
                           tag_in, cursor, perm, ptag);
        hipLaunchKernelGGL(k_sort_bricks, dim3((unsigned)std::min<int64_t>(nscan - 1, 1 << 20)),
                           dim3(kBrickSortThreads), 0, s, start, nscan - 1, ptag, perm);
        hipLaunchKernelGGL(k_sort_permute, dim3(grid_for(N)), dim3(kSortThreads), 0, s, perm, N,
                           reinterpret_cast<const float4*>(R_in), reinterpret_cast<const float4*>(V_in),
                           T_in, tag_in, reinterpret_cast<float4*>(R_out),
                           reinterpret_cast<float4*>(V_out), T_out, tag_out, inv);
        if (D > 0 && bonds_in)
            hipLaunchKernelGGL(k_sort_bonds, dim3(grid_for(N)), dim3(kSortThreads), 0, s, perm, inv,
                               N, bonds_in, D, bonds_out);
    }
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

}  // namespace hpf
