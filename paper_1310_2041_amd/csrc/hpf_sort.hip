// Canonical cell-list order of the beads (the paper reorders particle data for
// cache hits and bins beads into a cell list, Algorithm 1 Kernel 1).
//
// The key of a bead is the brick of B^3 cells holding its cell (one more key
// for beads that cannot be binned); the order is ascending (key, tag), where
// the tags are a permutation of [0, N) (the beads' original indices). Inside
// a brick the beads of a chain (consecutive tags) then stay neighbours, so
// most bond partners are adjacent in memory. The order is produced by a
// stable counting sort of the beads taken in tag order, so beads of one key
// come out in tag order with no sorting inside a key:
//   1. in storage order: idx[tag[i]] = i and key_t[tag[i]] = the key of bead i;
//   2. the tag sequence is cut into chunks of S tags; per chunk a key
//      histogram is counted in LDS and stored as one row of a chunk x key
//      table;
//   3. a column-wise exclusive scan of that table, taken in key-major order,
//      gives every (chunk, key) pair its first output slot, and the key
//      starts (cell_start);
//   4. per chunk the beads are placed in tag order: the lanes of a wavefront
//      that share a key take consecutive slots, and the wavefronts of a
//      workgroup take turns.
// No step needs a global atomic, and the result does not depend on the input
// order. Finally the bead arrays are gathered into the output buffers and the
// bond table is permuted and renumbered through the inverse permutation.
#include <algorithm>

#include "hpf_common.hpp"

namespace hpf {

struct SortK {
    MeshK m;
    int32_t B;
    int32_t nb[3];
    uint32_t NK;        // number of bricks; key NK = "cannot be binned"
};

constexpr int kSortThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kSortThreads * kScanPer;   // entries per scan block
constexpr int kScanTopThreads = 1024;
constexpr int kScanTopPer = 8;
constexpr int kMaxScanTiles = kScanTopThreads * kScanTopPer;
constexpr int kChunkThreads = 256;                    // histogram / placement workgroups
constexpr int kPlaceRegs = 16;                        // 256-tag blocks a thread holds at once
constexpr int64_t kMinChunk = (int64_t)kChunkThreads * kPlaceRegs;   // 4096 tags (one placement round)
constexpr int64_t kSmallChunk = kChunkThreads * 4;                    // 1024 tags
constexpr int64_t kChunksWanted = 2048;     // chunks that keep the histogram and placement passes busy
constexpr int kColBlock = 64;                         // chunks per column-scan block
constexpr int64_t kMaxSortKeys = 36864;               // one chunk's histogram in LDS (144 KiB)
constexpr int64_t kMaxTable = 64LL << 20;             // chunk x key table entries
constexpr uint32_t kNoKey = 0xffffffffu;              // a tag that names no bead

__global__ __launch_bounds__(kSortThreads) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kSortThreads)
        p[i] = v;
}

// ------------------------------------------------------------ scan (u32) --

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

// ------------------------------------------------------------------ keys --

// Sort key of bead i of one system.
struct CellKeyer {
    SortK sk;
    const float3* R;
    __device__ __forceinline__ uint32_t operator()(int32_t i) const
    {
        BeadCell b;
        return bead_cell(R[i], sk.m, b) ? brick_of(b.c[0], b.c[1], b.c[2], sk.B, sk.nb) : sk.NK;
    }
};

// ------------------------------------------ 1. tag -> index, and the keys --

// In storage order (coalesced reads of the positions): idx[tag] = i and key_t[tag] = the
// key of bead i. Tags missing from a broken permutation keep stale entries; the histogram
// pass finds them by idx < 0 (idx is filled with -1 first) and sets their key to none.
template <class Keyer>
__global__ __launch_bounds__(kSortThreads) void k_tag_index(Keyer keyer, const int32_t* __restrict__ tag,
                                                            int64_t N, int32_t* __restrict__ idx,
                                                            uint32_t* __restrict__ key_t)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * kSortThreads + threadIdx.x;
    if (i >= N)
        return;
    const int32_t t = tag ? tag[i] : (int32_t)i;
    if (t < 0 || t >= N) {
        raise_flag(HPF_FLAG_SORT_ORDER);
    } else {
        idx[t] = (int32_t)i;
        key_t[t] = keyer((int32_t)i);
    }
}

// ------------------------------------------------------ 2. chunk histograms --

__global__ __launch_bounds__(kChunkThreads) void k_sort_hist(const int32_t* __restrict__ idx,
                                                             int64_t N, int64_t S, uint32_t nkeys,
                                                             uint32_t* __restrict__ key_t,
                                                             uint32_t* __restrict__ table)
{
    extern __shared__ uint32_t hist[];
    const int64_t c = blockIdx.x;
    for (uint32_t k = threadIdx.x; k < nkeys; k += kChunkThreads)
        hist[k] = 0u;
    __syncthreads();
    const int64_t t0 = c * S, t1 = min(N, t0 + S);
    const int lane = threadIdx.x & (kWave - 1);
    bool missing = false;
    for (int64_t base = t0; base < t1; base += kChunkThreads) {
        const int64_t t = base + threadIdx.x;
        uint32_t key = kNoKey;
        if (t < t1) {
            if (idx[t] >= 0) {
                key = key_t[t];
            } else {
                missing = true;
                key_t[t] = kNoKey;
            }
        }
        const bool act = key != kNoKey;
        const uint64_t grp = wave_key_group(key, act);
        if (act && __builtin_ctzll(grp) == lane)
            atomicAdd(hist + key, (uint32_t)__builtin_popcountll(grp));
    }
    if (missing)
        raise_flag(HPF_FLAG_SORT_ORDER);
    __syncthreads();
    uint32_t* row = table + c * (int64_t)nkeys;
    for (uint32_t k = threadIdx.x; k < nkeys; k += kChunkThreads)
        row[k] = hist[k];
}

// ------------------------------------------------ 3. column-wise scan --

// part[cb][k] = sum of table[c][k] over the chunks c of column block cb
__global__ __launch_bounds__(kSortThreads) void k_col_partial(const uint32_t* __restrict__ table, int64_t nchunks,
                                                              uint32_t nkeys, uint32_t* __restrict__ part)
{
    const uint32_t k = blockIdx.x * kSortThreads + threadIdx.x;
    if (k >= nkeys)
        return;
    const int64_t c0 = (int64_t)blockIdx.y * kColBlock, c1 = min(nchunks, c0 + kColBlock);
    uint32_t s = 0;
    for (int64_t c = c0; c < c1; ++c)
        s += table[c * nkeys + k];
    part[(int64_t)blockIdx.y * nkeys + k] = s;
}

// part[cb][k] -> exclusive prefix over cb; tot[k] = key total
__global__ __launch_bounds__(kSortThreads) void k_col_prefix(uint32_t* __restrict__ part, int64_t ncb,
                                                             uint32_t nkeys, uint32_t* __restrict__ tot)
{
    const uint32_t k = blockIdx.x * kSortThreads + threadIdx.x;
    if (k >= nkeys)
        return;
    uint32_t run = 0;
    for (int64_t cb = 0; cb < ncb; ++cb) {
        const uint32_t v = part[cb * nkeys + k];
        part[cb * nkeys + k] = run;
        run += v;
    }
    tot[k] = run;
}

// table[c][k] -> first output slot of chunk c's beads with key k
__global__ __launch_bounds__(kSortThreads) void k_col_apply(uint32_t* __restrict__ table,
                                                            const uint32_t* __restrict__ part,
                                                            const uint32_t* __restrict__ start, int64_t nchunks,
                                                            uint32_t nkeys)
{
    const uint32_t k = blockIdx.x * kSortThreads + threadIdx.x;
    if (k >= nkeys)
        return;
    const int64_t c0 = (int64_t)blockIdx.y * kColBlock, c1 = min(nchunks, c0 + kColBlock);
    uint32_t run = start[k] + part[(int64_t)blockIdx.y * nkeys + k];
    for (int64_t c = c0; c < c1; ++c) {
        const uint32_t v = table[c * nkeys + k];
        table[c * nkeys + k] = run;
        run += v;
    }
}

// ------------------------------------------------------ 4. placement --

__global__ __launch_bounds__(kChunkThreads) void k_sort_place(const uint32_t* __restrict__ key_t,
                                                              const int32_t* __restrict__ idx, int64_t N, int64_t S,
                                                              uint32_t nkeys, const uint32_t* __restrict__ table,
                                                              int32_t* __restrict__ perm)
{
    extern __shared__ uint32_t next[];
    const int64_t c = blockIdx.x;
    const uint32_t* row = table + c * (int64_t)nkeys;
    for (uint32_t k = threadIdx.x; k < nkeys; k += kChunkThreads)
        next[k] = row[k];
    __syncthreads();
    const int64_t t0 = c * S, t1 = min(N, t0 + S);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int64_t g0 = t0; g0 < t1; g0 += kMinChunk) {
        uint32_t key[kPlaceRegs];
        int32_t src[kPlaceRegs];
        // 256-tag blocks of this round that hold tags (fewer than kPlaceRegs for a short chunk)
        const int nblk = (int)min((int64_t)kPlaceRegs, (t1 - g0 + kChunkThreads - 1) / kChunkThreads);
#pragma unroll
        for (int b = 0; b < kPlaceRegs; ++b) {
            const int64_t t = g0 + (int64_t)b * kChunkThreads + threadIdx.x;
            key[b] = kNoKey;
            src[b] = 0;
            if (t < t1) {
                key[b] = key_t[t];
                src[b] = idx[t];
            }
        }
#pragma unroll
        for (int b = 0; b < kPlaceRegs; ++b) {
            if (b >= nblk)                           // uniform: the block holds no tags
                continue;
            for (int w = 0; w < kChunkThreads / kWave; ++w) {
                if (wave == w) {
                    const bool act = key[b] != kNoKey;
                    const uint64_t grp = wave_key_group(key[b], act);
                    const int leader = act ? __builtin_ctzll(grp) : lane;
                    uint32_t base = 0;
                    if (act && leader == lane) {
                        base = next[key[b]];
                        next[key[b]] = base + (uint32_t)__builtin_popcountll(grp);
                    }
                    base = __shfl(base, leader, kWave);
                    if (act)
                        perm[base + (uint32_t)__builtin_popcountll(grp & ((1ull << lane) - 1))] = src[b];
                }
                __syncthreads();
            }
        }
    }
}

__global__ __launch_bounds__(kSortThreads) void k_iota(int32_t* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
    if (i < n)
        p[i] = (int32_t)i;
}

// ------------------------------------------------ gather and bond table --

__global__ __launch_bounds__(kSortThreads) void k_sort_permute(const int32_t* __restrict__ perm, int64_t N,
                                                               const float3* __restrict__ R_in,
                                                               const float3* __restrict__ V_in,
                                                               const uint8_t* __restrict__ T_in,
                                                               const int32_t* __restrict__ tag_in,
                                                               float3* __restrict__ R_out,
                                                               float3* __restrict__ V_out,
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

// Per-bead angle table in the new order: partner rows (3a, 3a + 1) renumbered
// like the bond table, code rows (3a + 2) moved with their bead unchanged.
__global__ __launch_bounds__(kSortThreads) void k_sort_angles(const int32_t* __restrict__ perm,
                                                              const int32_t* __restrict__ inv, int64_t N,
                                                              const int32_t* __restrict__ ang_in, int A,
                                                              int32_t* __restrict__ ang_out)
{
    const int64_t p = xcd_block(blockIdx.x, gridDim.x) * kSortThreads + threadIdx.x;
    if (p >= N)
        return;
    const int32_t o = perm[p];
    bool bad = false;
    for (int r = 0; r < 3 * A; ++r) {
        const int32_t j = ang_in[(int64_t)r * N + o];
        int32_t nj = j;
        if (r % 3 != 2) {
            nj = -1;
            if (j >= 0 && j < N)
                nj = inv[j];
            else if (j >= N || j < -1)
                bad = true;
        }
        ang_out[(int64_t)r * N + p] = nj;
    }
    if (bad)
        raise_flag(HPF_FLAG_BAD_BOND);
}

// ------------------------------------------- re-sort from a previous order --
//
// Between sorts most beads stay in their brick. When the input is in the order an
// earlier sort produced (ascending (key, tag) for the positions of that time) and
// that sort's key starts are given, the new order is built per key instead of over
// the whole tag sequence:
//   1. per old key range, in storage order (coalesced): every bead's new key; the
//      beads that keep their key ("stayers") are compacted in place, still in tag
//      order; the others ("movers") are counted per new key;
//   2. one scan gives the new key starts and each key's slot range for its movers;
//   3. every mover is appended (tag, index) to its new key's slots;
//   4. per new key: its movers are sorted by tag, and the stayers and the movers
//      are merged by tag: an element's position is its rank in its own list plus
//      the number of elements of the other list with a smaller tag (a binary
//      search).
// The result equals the stable counting sort's exactly: (key, tag) order.
constexpr int kResortThreads = 256;
constexpr int kPlaceThreads = 512;
constexpr int kMoverCap = 4096;          // movers of one key sorted in LDS (32 KiB)

__device__ __forceinline__ int32_t tag_of(const int32_t* __restrict__ tag, int64_t i)
{
    return tag ? tag[i] : (int32_t)i;
}

template <class Keyer>
__global__ __launch_bounds__(kResortThreads) void k_resort_keys(Keyer keyer, const int32_t* __restrict__ tag,
                                                                const uint32_t* __restrict__ cs_old, int64_t N,
                                                                uint32_t* __restrict__ keyp,
                                                                int32_t* __restrict__ stayidx,
                                                                uint32_t* __restrict__ cnt_stay,
                                                                uint32_t* __restrict__ cnt_move)
{
    __shared__ uint32_t sh[kResortThreads / kWave + 1];
    const uint32_t k = blockIdx.x;
    const int64_t a = min((int64_t)cs_old[k], N), b = min((int64_t)cs_old[k + 1], N);
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t run = 0;
    bool bad = false;
    for (int64_t base = a; base < b; base += kResortThreads) {
        const int64_t i = base + threadIdx.x;
        uint32_t key = kNoKey;
        if (i < b) {
            key = keyer((int32_t)i);
            keyp[i] = key;
            // the precondition: every old key range in ascending tag order
            bad |= i > a && tag_of(tag, i) <= tag_of(tag, i - 1);
        }
        const bool stay = key == k;
        uint32_t total;
        const uint32_t r = block_excl_scan<kResortThreads>(stay ? 1u : 0u, sh, &total);
        if (stay)
            stayidx[a + run + r] = (int32_t)i;
        run += total;
        const bool mv = i < b && !stay;
        const uint64_t grp = wave_key_group(key, mv);
        if (mv && __builtin_ctzll(grp) == lane)
            atomicAdd(cnt_move + key, (uint32_t)__builtin_popcountll(grp));
    }
    if (threadIdx.x == 0)
        cnt_stay[k] = run;
    if (bad)
        raise_flag(HPF_FLAG_SORT_ORDER);
}

// One block: new key starts (stayers + movers per key, exclusive scan; the last entry
// the total) and the movers' slot offsets (exclusive scan of the mover counts); the
// slot fill counters are cleared.
constexpr int kResortScanThreads = 1024;

__global__ __launch_bounds__(kResortScanThreads) void k_resort_scan(const uint32_t* __restrict__ cnt_stay,
                                                                    const uint32_t* __restrict__ cnt_move,
                                                                    uint32_t nkeys, uint32_t* __restrict__ start,
                                                                    uint32_t* __restrict__ moff,
                                                                    uint32_t* __restrict__ fill)
{
    __shared__ uint32_t sh[kResortScanThreads / kWave + 1];
    const uint32_t per = (nkeys + kResortScanThreads - 1) / kResortScanThreads;
    const uint32_t k0 = min(nkeys, threadIdx.x * per), k1 = min(nkeys, k0 + per);
    uint32_t st = 0, mv = 0;
    for (uint32_t k = k0; k < k1; ++k) {
        st += cnt_stay[k] + cnt_move[k];
        mv += cnt_move[k];
    }
    uint32_t tot_st, tot_mv;
    uint32_t run_st = block_excl_scan<kResortScanThreads>(st, sh, &tot_st);
    uint32_t run_mv = block_excl_scan<kResortScanThreads>(mv, sh, &tot_mv);
    for (uint32_t k = k0; k < k1; ++k) {
        start[k] = run_st;
        moff[k] = run_mv;
        fill[k] = 0u;
        run_st += cnt_stay[k] + cnt_move[k];
        run_mv += cnt_move[k];
    }
    if (threadIdx.x == 0) {
        start[nkeys] = tot_st;
        moff[nkeys] = tot_mv;
    }
}

// Movers appended to their new key's slots as (tag << 32 | index); their order inside
// a key's slots is arbitrary (sorted in the placement).
__global__ __launch_bounds__(kResortThreads) void k_resort_movers(const int32_t* __restrict__ tag,
                                                                  const uint32_t* __restrict__ cs_old, int64_t N,
                                                                  const uint32_t* __restrict__ keyp,
                                                                  const uint32_t* __restrict__ moff,
                                                                  uint32_t* __restrict__ fill,
                                                                  unsigned long long* __restrict__ movers)
{
    const uint32_t k = blockIdx.x;
    const int64_t a = min((int64_t)cs_old[k], N), b = min((int64_t)cs_old[k + 1], N);
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t base = a; base < b; base += kResortThreads) {
        const int64_t i = base + threadIdx.x;
        const uint32_t key = i < b ? keyp[i] : kNoKey;
        const bool mv = i < b && key != k;
        const uint64_t grp = wave_key_group(key, mv);
        const int leader = mv ? __builtin_ctzll(grp) : lane;
        uint32_t slot = 0;
        if (mv && leader == lane)
            slot = atomicAdd(fill + key, (uint32_t)__builtin_popcountll(grp));
        slot = __shfl(slot, leader, kWave);
        if (mv) {
            slot += (uint32_t)__builtin_popcountll(grp & ((1ull << lane) - 1));
            movers[(int64_t)moff[key] + slot] =
                ((unsigned long long)(uint32_t)tag_of(tag, i) << 32) | (unsigned long long)(uint32_t)i;
        }
    }
}

// Ascending sort of v[0, n) padded with +inf to p (a power of two): a bitonic network
// whose comparators all put the smaller value first (the first step of every merge
// compares mirrored positions), so the padding never moves forward. All threads call.
template <class Load, class Store>
__device__ __forceinline__ void sort_padded(int64_t n, int64_t p, Load load, Store store)
{
    for (int64_t size = 2; size <= p; size <<= 1) {
        for (int64_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int64_t q = threadIdx.x; q < p / 2; q += blockDim.x) {
                // the q-th comparator of this step: elements i < j
                const int64_t blk = q / stride, off = q % stride;
                int64_t i = blk * 2 * stride + off, j = i + stride;
                if (stride == (size >> 1))
                    j = (i / size) * size + size - 1 - (i % size);   // mirrored partner
                if (j < n) {
                    const unsigned long long a = load(i), c = load(j);
                    if (c < a) {
                        store(i, c);
                        store(j, a);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Per new key: movers sorted by tag (in LDS when they fit, else in place in their
// slots), then stayers and movers merged by tag into the key's output range.
__global__ __launch_bounds__(kPlaceThreads) void k_resort_place(const int32_t* __restrict__ tag,
                                                                const uint32_t* __restrict__ cs_old, int64_t N,
                                                                const int32_t* __restrict__ stayidx,
                                                                const uint32_t* __restrict__ cnt_stay,
                                                                const uint32_t* __restrict__ cnt_move,
                                                                const uint32_t* __restrict__ moff,
                                                                const uint32_t* __restrict__ start,
                                                                unsigned long long* __restrict__ movers,
                                                                int32_t* __restrict__ perm)
{
    __shared__ unsigned long long smv[kMoverCap];
    const uint32_t k = blockIdx.x;
    const int64_t nmv = cnt_move[k], ns = cnt_stay[k];
    const int64_t base = start[k];
    unsigned long long* mv = movers + moff[k];
    const int32_t* st = stayidx + min((int64_t)cs_old[k], N);
    int64_t p2 = 1;
    while (p2 < nmv)
        p2 <<= 1;
    const bool in_lds = nmv <= kMoverCap;
    if (in_lds) {
        for (int64_t q = threadIdx.x; q < nmv; q += kPlaceThreads)
            smv[q] = mv[q];
        __syncthreads();
        sort_padded(nmv, p2, [&](int64_t q) { return smv[q]; }, [&](int64_t q, unsigned long long v) { smv[q] = v; });
    } else {
        sort_padded(nmv, p2, [&](int64_t q) { return mv[q]; }, [&](int64_t q, unsigned long long v) { mv[q] = v; });
    }
    // movers: rank among movers + stayers with a smaller tag
    for (int64_t q = threadIdx.x; q < nmv; q += kPlaceThreads) {
        const unsigned long long e = in_lds ? smv[q] : mv[q];
        const int32_t t = (int32_t)(e >> 32);
        int64_t lo = 0, hi = ns;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (tag_of(tag, st[mid]) < t)
                lo = mid + 1;
            else
                hi = mid;
        }
        perm[base + q + lo] = (int32_t)(uint32_t)e;
    }
    // stayers: rank among stayers + movers with a smaller tag
    for (int64_t q = threadIdx.x; q < ns; q += kPlaceThreads) {
        const int32_t i = st[q];
        const unsigned long long t = (unsigned long long)(uint32_t)tag_of(tag, i) << 32;
        int64_t lo = 0, hi = nmv;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((in_lds ? smv[mid] : mv[mid]) < t)
                lo = mid + 1;
            else
                hi = mid;
        }
        perm[base + q + lo] = i;
    }
}

// ------------------------------------------------------------------ host --

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Sizes and workspace layout of one sort of N beads over nkeys keys.
struct SortPlan {
    int64_t N = 0;
    uint32_t nkeys = 0;
    int64_t S = 0, nchunks = 0, ncb = 0, nscan = 0, ntiles = 0;
    size_t off_key = 0, off_perm = 0, off_idx = 0, off_table = 0, off_part = 0, off_tiles = 0, off_start = 0;
    // re-sort from a previous order: compacted stayers, movers, per-key counts and offsets
    size_t off_stay = 0, off_movers = 0, off_cstay = 0, off_cmove = 0, off_fill = 0, off_moff = 0;
    size_t bytes = 0;
};

bool sort_plan(int64_t N, int64_t nkeys, SortPlan* p)
{
    if (N < 0 || N > 0x7ffffff0LL || nkeys < 1 || nkeys > kMaxSortKeys)
        return false;
    // Chunks of 4096 tags (one placement round), or of 1024 when that leaves fewer
    // than kChunksWanted chunks and the chunk x key table stays within 4 entries
    // per bead; larger while the table exceeds kMaxTable.
    int64_t S = kMinChunk;
    if ((N + S - 1) / S < kChunksWanted && ((N + kSmallChunk - 1) / kSmallChunk) * nkeys <= 4 * std::max<int64_t>(N, 1))
        S = kSmallChunk;
    while (((N + S - 1) / S) * nkeys > kMaxTable)
        S *= 2;
    p->N = N;
    p->nkeys = (uint32_t)nkeys;
    p->S = S;
    p->nchunks = std::max<int64_t>(1, (N + S - 1) / S);
    p->ncb = (p->nchunks + kColBlock - 1) / kColBlock;
    p->nscan = nkeys + 1;
    p->ntiles = (p->nscan + kScanTile - 1) / kScanTile;
    if (p->ntiles > kMaxScanTiles)
        return false;
    const size_t N1 = (size_t)(N > 0 ? N : 1);
    size_t o = 0;
    p->off_key = o; o += align_up(sizeof(uint32_t) * N1);
    p->off_perm = o; o += align_up(sizeof(int32_t) * N1);
    p->off_idx = o; o += align_up(sizeof(int32_t) * N1);          // tag index, then inverse permutation
    p->off_table = o; o += align_up(sizeof(uint32_t) * (size_t)p->nchunks * (size_t)nkeys);
    p->off_part = o; o += align_up(sizeof(uint32_t) * (size_t)p->ncb * (size_t)nkeys);
    p->off_tiles = o; o += align_up(sizeof(uint32_t) * (size_t)(p->ntiles + 1));
    p->off_start = o; o += align_up(sizeof(uint32_t) * (size_t)(p->nscan + 1));
    p->off_stay = o; o += align_up(sizeof(int32_t) * N1);
    p->off_movers = o; o += align_up(sizeof(uint64_t) * N1);
    p->off_cstay = o; o += align_up(sizeof(uint32_t) * (size_t)nkeys);
    p->off_cmove = o; o += align_up(sizeof(uint32_t) * (size_t)nkeys);
    p->off_fill = o; o += align_up(sizeof(uint32_t) * (size_t)nkeys);
    p->off_moff = o; o += align_up(sizeof(uint32_t) * (size_t)(nkeys + 1));
    p->bytes = o;
    return true;
}

bool sort_layout(int64_t N, const int32_t M[3], int B, SortK* sk_out, SortPlan* plan)
{
    if (B == 0)
        B = 8;
    if (B < 1 || B > 16)
        return false;
    int64_t nk = 1;
    int32_t nb[3];
    for (int d = 0; d < 3; ++d) {
        nb[d] = (M[d] + B - 1) / B;
        nk *= nb[d];
    }
    if (!sort_plan(N, nk + 1, plan))
        return false;
    if (sk_out) {
        sk_out->B = B;
        for (int d = 0; d < 3; ++d)
            sk_out->nb[d] = nb[d];
        sk_out->NK = (uint32_t)nk;
    }
    return true;
}

static unsigned grid_for(int64_t n) { return (unsigned)((n + kSortThreads - 1) / kSortThreads); }

// The four steps and the gather for any key function; `start` receives the
// key starts (nkeys + 1 entries, the last = number of placed beads).
template <class Keyer>
hpf_status_t run_sort(const SortPlan& pl, Keyer keyer, int64_t N, const float* R_in, const float* V_in,
                      const uint8_t* T_in, const int32_t* tag_in, const int32_t* bonds_in, int D, float* R_out,
                      float* V_out, uint8_t* T_out, int32_t* tag_out, int32_t* bonds_out, uint32_t* start,
                      char* work, hipStream_t s)
{
    uint32_t* key_t = reinterpret_cast<uint32_t*>(work + pl.off_key);
    int32_t* perm = reinterpret_cast<int32_t*>(work + pl.off_perm);
    int32_t* idx = reinterpret_cast<int32_t*>(work + pl.off_idx);
    uint32_t* table = reinterpret_cast<uint32_t*>(work + pl.off_table);
    uint32_t* part = reinterpret_cast<uint32_t*>(work + pl.off_part);
    uint32_t* tiles = reinterpret_cast<uint32_t*>(work + pl.off_tiles);
    const uint32_t nk = pl.nkeys;
    const size_t smem = sizeof(uint32_t) * nk;
    if (smem > 65536 &&
        (hipFuncSetAttribute(reinterpret_cast<const void*>(k_sort_hist),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess ||
         hipFuncSetAttribute(reinterpret_cast<const void*>(k_sort_place), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)smem) != hipSuccess))
        return HPF_EINVAL;
    const unsigned gfill = (unsigned)std::min<int64_t>(grid_for(pl.nscan), 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(gfill), dim3(kSortThreads), 0, s, start, pl.nscan, 0u);
    if (N > 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>(grid_for(N), 4096)), dim3(kSortThreads), 0, s,
                           reinterpret_cast<uint32_t*>(idx), N, 0xffffffffu);
        hipLaunchKernelGGL(k_iota, dim3(grid_for(N)), dim3(kSortThreads), 0, s, perm, N);
        hipLaunchKernelGGL(k_tag_index<Keyer>, dim3(grid_for(N)), dim3(kSortThreads), 0, s, keyer, tag_in, N, idx,
                           key_t);
        hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)pl.nchunks), dim3(kChunkThreads), smem, s, idx,
                           N, pl.S, nk, key_t, table);
        const dim3 gcol((nk + kSortThreads - 1) / kSortThreads, (unsigned)pl.ncb);
        hipLaunchKernelGGL(k_col_partial, gcol, dim3(kSortThreads), 0, s, table, pl.nchunks, nk, part);
        hipLaunchKernelGGL(k_col_prefix, dim3((nk + kSortThreads - 1) / kSortThreads), dim3(kSortThreads), 0, s,
                           part, pl.ncb, nk, start);
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)pl.ntiles), dim3(kSortThreads), 0, s, start, pl.nscan, tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTopThreads), 0, s, tiles, (int)pl.ntiles);
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(pl.nscan)), dim3(kSortThreads), 0, s, start, pl.nscan, tiles);
    if (N > 0) {
        const dim3 gcol((nk + kSortThreads - 1) / kSortThreads, (unsigned)pl.ncb);
        hipLaunchKernelGGL(k_col_apply, gcol, dim3(kSortThreads), 0, s, table, part, start, pl.nchunks, nk);
        hipLaunchKernelGGL(k_sort_place, dim3((unsigned)pl.nchunks), dim3(kChunkThreads), smem, s, key_t, idx, N,
                           pl.S, nk, table, perm);
        hipLaunchKernelGGL(k_sort_permute, dim3(grid_for(N)), dim3(kSortThreads), 0, s, perm, N,
                           reinterpret_cast<const float3*>(R_in), reinterpret_cast<const float3*>(V_in), T_in,
                           tag_in, reinterpret_cast<float3*>(R_out), reinterpret_cast<float3*>(V_out), T_out,
                           tag_out, idx);
        if (D > 0 && bonds_in)
            hipLaunchKernelGGL(k_sort_bonds, dim3(grid_for(N)), dim3(kSortThreads), 0, s, perm, idx, N, bonds_in,
                               D, bonds_out);
    }
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t launch_sort(const SortK& sk, const SortPlan& pl, int64_t N, const float* R_in, const float* V_in,
                         const uint8_t* T_in, const int32_t* tag_in, const int32_t* bonds_in, int D, float* R_out,
                         float* V_out, uint8_t* T_out, int32_t* tag_out, int32_t* bonds_out, uint32_t* cell_start,
                         char* work, hipStream_t s)
{
    CellKeyer keyer{sk, reinterpret_cast<const float3*>(R_in)};
    uint32_t* start = cell_start ? cell_start : reinterpret_cast<uint32_t*>(work + pl.off_start);
    return run_sort(pl, keyer, N, R_in, V_in, T_in, tag_in, bonds_in, D, R_out, V_out, T_out, tag_out, bonds_out,
                    start, work, s);
}

// The re-sort (steps 1-4 above), then the gather and the bond renumbering of run_sort.
hpf_status_t launch_resort(const SortK& sk, const SortPlan& pl, int64_t N, const float* R_in, const float* V_in,
                           const uint8_t* T_in, const int32_t* tag_in, const int32_t* bonds_in, int D, float* R_out,
                           float* V_out, uint8_t* T_out, int32_t* tag_out, int32_t* bonds_out,
                           const uint32_t* cs_old, uint32_t* cs_new, char* work, hipStream_t s)
{
    CellKeyer keyer{sk, reinterpret_cast<const float3*>(R_in)};
    const uint32_t nk = pl.nkeys;
    auto* keyp = reinterpret_cast<uint32_t*>(work + pl.off_key);
    auto* perm = reinterpret_cast<int32_t*>(work + pl.off_perm);
    auto* inv = reinterpret_cast<int32_t*>(work + pl.off_idx);
    auto* stay = reinterpret_cast<int32_t*>(work + pl.off_stay);
    auto* movers = reinterpret_cast<unsigned long long*>(work + pl.off_movers);
    auto* cstay = reinterpret_cast<uint32_t*>(work + pl.off_cstay);
    auto* cmove = reinterpret_cast<uint32_t*>(work + pl.off_cmove);
    auto* fill = reinterpret_cast<uint32_t*>(work + pl.off_fill);
    auto* moff = reinterpret_cast<uint32_t*>(work + pl.off_moff);
    const unsigned gfill = (unsigned)std::min<int64_t>(grid_for(nk), 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(gfill), dim3(kSortThreads), 0, s, cmove, (int64_t)nk, 0u);
    if (N > 0) {
        // every output slot holds a valid index even if the input breaks the precondition
        hipLaunchKernelGGL(k_iota, dim3(grid_for(N)), dim3(kSortThreads), 0, s, perm, N);
        hipLaunchKernelGGL(k_resort_keys<CellKeyer>, dim3(nk), dim3(kResortThreads), 0, s, keyer, tag_in, cs_old, N,
                           keyp, stay, cstay, cmove);
    } else {
        hipLaunchKernelGGL(k_fill_u32, dim3(gfill), dim3(kSortThreads), 0, s, cstay, (int64_t)nk, 0u);
    }
    hipLaunchKernelGGL(k_resort_scan, dim3(1), dim3(kResortScanThreads), 0, s, cstay, cmove, nk, cs_new, moff, fill);
    if (N > 0) {
        hipLaunchKernelGGL(k_resort_movers, dim3(nk), dim3(kResortThreads), 0, s, tag_in, cs_old, N, keyp, moff, fill,
                           movers);
        hipLaunchKernelGGL(k_resort_place, dim3(nk), dim3(kPlaceThreads), 0, s, tag_in, cs_old, N, stay, cstay, cmove,
                           moff, cs_new, movers, perm);
        hipLaunchKernelGGL(k_sort_permute, dim3(grid_for(N)), dim3(kSortThreads), 0, s, perm, N,
                           reinterpret_cast<const float3*>(R_in), reinterpret_cast<const float3*>(V_in), T_in,
                           tag_in, reinterpret_cast<float3*>(R_out), reinterpret_cast<float3*>(V_out), T_out,
                           tag_out, inv);
        if (D > 0 && bonds_in)
            hipLaunchKernelGGL(k_sort_bonds, dim3(grid_for(N)), dim3(kSortThreads), 0, s, perm, inv, N, bonds_in,
                               D, bonds_out);
    }
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t launch_sort_angles(const SortPlan& pl, int64_t N, const int32_t* ang_in, int A, int32_t* ang_out,
                                const char* work, hipStream_t s)
{
    if (N == 0 || A == 0)
        return HPF_OK;
    const int32_t* perm = reinterpret_cast<const int32_t*>(work + pl.off_perm);
    const int32_t* inv = reinterpret_cast<const int32_t*>(work + pl.off_idx);
    hipLaunchKernelGGL(k_sort_angles, dim3(grid_for(N)), dim3(kSortThreads), 0, s, perm, inv, N, ang_in, A, ang_out);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

}  // namespace hpf
