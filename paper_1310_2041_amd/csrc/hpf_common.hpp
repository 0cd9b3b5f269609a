// Internal device helpers of libhpf (gfx950, wave64). Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <tuple>

#include "hpf.h"

namespace hpf {

constexpr int kWave = 64;
constexpr uint32_t kOne = 1u << HPF_FIX_BITS;          // 2^S
constexpr float kInvOne = 1.0f / 65536.0f;              // 2^-S, exact

// Sticky device status word (one per device); read by hpf_get_device_status.
extern __device__ uint32_t g_status;

__device__ __forceinline__ void raise_flag(uint32_t bit) { atomicOr(&g_status, bit); }

// Mesh description as passed to kernels (by value).
struct MeshK {
    float L[3];
    float halfL[3];
    float s[3];
    int32_t M[3];
    int64_t nm;         // Mx * My * Mz
    double c_norm;
};

// Cell index and upper 1-D fixed-point weight of one coordinate.
// u = fl32(x * s) (single rounding, no contraction), c = floor(u) mod M,
// f = fl32(u - floor(u)), q = floor(f * 2^S). The lower weight is 2^S - q.
// Returns false for a coordinate that cannot be binned (non-finite or
// |u| >= 2^24).
__device__ __forceinline__ bool cell_coord(float x, float s, int32_t M, int32_t& c, uint32_t& q)
{
    const float u = __fmul_rn(x, s);
    if (!(fabsf(u) < 16777216.0f))
        return false;
    const float fl = floorf(u);
    const float f = __fsub_rn(u, fl);
    q = (uint32_t)__fmul_rn(f, 65536.0f);
    int32_t ci = (int32_t)fl;
    if ((uint32_t)ci >= (uint32_t)M) {
        ci %= M;
        if (ci < 0)
            ci += M;
    }
    c = ci;
    return true;
}

struct BeadCell {
    int32_t c[3];
    uint32_t q[3];
};

__device__ __forceinline__ bool bead_cell(const float3& r, const MeshK& m, BeadCell& b)
{
    bool ok = cell_coord(r.x, m.s[0], m.M[0], b.c[0], b.q[0]);
    ok = cell_coord(r.y, m.s[1], m.M[1], b.c[1], b.q[1]) && ok;
    ok = cell_coord(r.z, m.s[2], m.M[2], b.c[2], b.q[2]) && ok;
    return ok;
}

// Streaming accesses: data that a pass reads or writes once (its own bead rows, the
// bond table, the stored deposit boxes) go through the caches with the nontemporal
// hint, so that their lines are the first evicted and the gradient mesh and the bond
// partners, which are read many times, stay in L2.
__device__ __forceinline__ float3 load_stream(const float3* p)
{
    const float* q = reinterpret_cast<const float*>(p);
    return make_float3(__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1),
                       __builtin_nontemporal_load(q + 2));
}
__device__ __forceinline__ void store_stream(float3* p, const float3& v)
{
    float* q = reinterpret_cast<float*>(p);
    __builtin_nontemporal_store(v.x, q);
    __builtin_nontemporal_store(v.y, q + 1);
    __builtin_nontemporal_store(v.z, q + 2);
}
template <class T>
__device__ __forceinline__ T load_stream(const T* p)
{
    return __builtin_nontemporal_load(p);
}
template <class T>
__device__ __forceinline__ void store_stream(T* p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// kNT selects the hint. It pays only where a pass streams more than the 256 MB Infinity
// Cache keeps from one step to the next; on smaller systems the next step finds the bead
// rows there, and the hint would push them out.
template <bool kNT, class T>
__device__ __forceinline__ T load_hint(const T* p)
{
    if constexpr (kNT)
        return load_stream(p);
    else
        return *p;
}
template <bool kNT, class T>
__device__ __forceinline__ void store_hint(T* p, const T& v)
{
    if constexpr (kNT)
        store_stream(p, v);
    else
        *p = v;
}
// Bytes a fused pass streams above which it takes the hint: half the Infinity Cache, as the
// step also reads and writes the mesh arrays and the other position buffer.
constexpr int64_t kStreamHintBytes = int64_t(128) << 20;

__device__ __forceinline__ int32_t next_wrap(int32_t c, int32_t M) { return c + 1 == M ? 0 : c + 1; }
__device__ __forceinline__ int32_t prev_wrap(int32_t c, int32_t M) { return c == 0 ? M - 1 : c - 1; }

// Workgroups are dispatched round-robin over the 8 XCDs (WG b on XCD b % 8).
// Map them so that each XCD works on one contiguous range of logical blocks:
// neighbouring tiles then share that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks)
{
    const int64_t per = nblocks >> 3, rem = nblocks & 7;
    const int64_t xcd = b & 7, idx = b >> 3;
    const int64_t base = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return base + idx;
}

// Work split of a persistent grid over n items (bricks): the items are cut
// into one contiguous run per XCD (workgroup b runs on XCD b % 8), and that
// XCD's workgroups take the items of its run in turn, so the items in flight
// at any moment are neighbours.
struct BrickWalk {
    int64_t end, first, stride;
};

__device__ __forceinline__ BrickWalk brick_walk(int64_t n)
{
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t ng = nb < 8 ? nb : 8;
    const int64_t g = b % ng, idx = b / ng;
    const int64_t per_group = nb / ng + (g < nb % ng ? 1 : 0);
    BrickWalk w;
    w.first = n * g / ng + idx;
    w.end = n * (g + 1) / ng;
    w.stride = per_group;
    return w;
}

// Fixed-order wave64 sum (butterfly), identical result in every lane.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    return v;
}

// Fixed-order block sum of one double per thread. `scratch` holds one double
// per wave. Result valid in thread 0. blockDim.x must be a multiple of 64.
__device__ __forceinline__ double block_sum(double v, double* scratch)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0)
        scratch[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / kWave;
        for (int w = 0; w < nw; ++w)
            t += scratch[w];
    }
    __syncthreads();
    return t;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = min(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

// Inclusive wave64 scan.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(v, off, kWave);
        if (lane >= off)
            v += t;
    }
    return v;
}

// Exclusive block scan of one value per thread; returns the exclusive prefix
// and the block total through *total.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1)
        sh[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < NT / kWave; ++w) {
            const uint32_t t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[NT / kWave] = run;
    }
    __syncthreads();
    const uint32_t r = sh[wid] + inc - v;
    *total = sh[NT / kWave];
    __syncthreads();
    return r;
}

// Lanes of a wavefront grouped by equal key, whatever their positions: one
// pass per distinct key among the active lanes (a uniform loop). Returns the
// mask of active lanes holding this lane's key (0 for inactive lanes); its
// lowest set bit is the group's leader, popcount its size, and the bits below
// this lane give its rank in the group.
__device__ __forceinline__ uint64_t wave_key_group(uint32_t key, bool active)
{
    uint64_t remaining = __ballot(active);
    uint64_t mine = 0;
    while (remaining) {
        const int leader = __builtin_ctzll(remaining);
        const uint32_t k = __shfl(key, leader, kWave);
        const uint64_t m = __ballot(active && key == k);
        if (active && key == k)
            mine = m;
        remaining &= ~m;
    }
    return mine;
}

// Minimum-image separation x_j - x_i along one axis of a periodic box for
// coordinates inside [0, L). When the raw difference exceeds half a box the
// wrapped coordinate is formed first (x_j - L or x_i - L is exact by Sterbenz's
// lemma), so the result carries a rounding error of the short bond vector
// rather than of the box length. Far-away inputs fall back to rint.
__device__ __forceinline__ float min_image(float xj, float xi, float L, float halfL)
{
    float d = xj - xi;
    if (fabsf(d) > halfL) {
        if (fabsf(d) < 1.5f * L)
            d = d > 0.0f ? (xj - L) - xi : xj - (xi - L);
        else
            d = d - L * rintf(d / L);
    }
    return d;
}

// Wrap a coordinate into [0, L): fmod is exact; a result that rounds up to L
// after adding L becomes 0.
__device__ __forceinline__ float wrap_coord(float x, float L)
{
    if (x >= 0.0f && x < L)
        return x;
    float r = fmodf(x, L);
    if (r < 0.0f)
        r += L;
    if (r >= L)
        r = 0.0f;
    return r;
}

// Workgroups of `fn` (with `threads` threads and `smem` bytes of dynamic LDS)
// that the current device holds at once: blocks per CU from the occupancy
// calculator (registers and LDS) times the CU count. Cached per device and
// shape; 0 if the runtime cannot tell.
inline int64_t resident_blocks(const void* fn, int threads, size_t smem)
{
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, int, size_t>, int64_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0;
    const auto key = std::make_tuple(dev, fn, threads, smem);
    std::lock_guard<std::mutex> lock(mu);
    const auto it = cache.find(key);
    if (it != cache.end())
        return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, smem) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int64_t n = (int64_t)per_cu * cus;
    cache[key] = n;
    return n;
}

}  // namespace hpf
