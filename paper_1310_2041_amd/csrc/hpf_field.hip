// Mesh-side kernels: the external potential of eq. (4) from the fixed-point
// counts, and its centred periodic gradient (Algorithm 1 Kernel 3, read as a
// centred difference at the mesh point). Both are streaming, HBM-bound
// passes over the mesh.
#include <algorithm>

#include "hpf_common.hpp"

namespace hpf {

struct PotK {
    double A[HPF_MAX_TYPES * HPF_MAX_TYPES];   // kT * chi, row-major K x K
    double inv_kappa;
    double rho0_dV;                            // N / (Mx My Mz), scales the energy
};

constexpr int kPotThreads = 256;

// Potential at mesh point q of one system: phi_K = n_K c_norm in FP64,
// V_K = sum_K' A_KK' phi_K' + inv_kappa (sum phi - 1) stored as FP32, counts
// cleared for the next scatter. Returns the point's field-energy term
// (without the rho0 dV factor).
// The same from counts n[K] already in registers (V written, nothing cleared).
template <int K>
__device__ __forceinline__ double potential_values(const unsigned long long (&n)[K], float* __restrict__ V,
                                                   int64_t nm, int64_t q, double c_norm, const PotK& p, bool& over)
{
    double phi[K];
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        over |= n[k] >= (1ull << 62);
        phi[k] = (double)n[k] * c_norm;
        tot += phi[k];
    }
    const double delta = tot - 1.0;
    double inter = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double mix = 0.0;
#pragma unroll
        for (int kk = 0; kk < K; ++kk)
            mix += p.A[k * K + kk] * phi[kk];
        V[k * nm + q] = (float)(mix + p.inv_kappa * delta);
        inter += phi[k] * mix;
    }
    return 0.5 * inter + 0.5 * p.inv_kappa * delta * delta;
}

// Composition list of a mesh point (the paper's list of the species with a
// non-zero density there, used to shorten the species loop): bit k set when
// species k has a non-zero count.
template <int K>
__device__ __forceinline__ uint8_t composition(const unsigned long long (&n)[K])
{
    uint32_t bits = 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        bits |= (n[k] != 0ull ? 1u : 0u) << k;
    return (uint8_t)bits;
}

template <int K>
__device__ __forceinline__ double potential_point(unsigned long long* __restrict__ counts,
                                                  float* __restrict__ V, int64_t nm, int64_t q,
                                                  double c_norm, const PotK& p, bool& over,
                                                  uint8_t* __restrict__ present)
{
    unsigned long long n[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        n[k] = counts[k * nm + q];
#pragma unroll
    for (int k = 0; k < K; ++k)
        counts[k * nm + q] = 0ull;
    if (present)
        present[q] = composition<K>(n);
    return potential_values<K>(n, V, nm, q, c_norm, p, over);
}

// One thread per mesh point (grid-stride); optional FP64 field-energy partials.
template <int K>
__global__ __launch_bounds__(kPotThreads) void k_field_potential(unsigned long long* __restrict__ counts,
                                                                 MeshK m, PotK p,
                                                                 float* __restrict__ V,
                                                                 double* __restrict__ w_part,
                                                                 uint8_t* __restrict__ present)
{
    __shared__ double scratch[kPotThreads / kWave];
    const int64_t nm = m.nm;
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    double wsum = 0.0;
    bool over = false;
    if (w_part)                                    // slots beyond this grid read as zero
        for (int64_t i = (int64_t)gridDim.x + blockIdx.x + (int64_t)threadIdx.x * gridDim.x; i < HPF_NPART;
             i += (int64_t)kPotThreads * gridDim.x)
            w_part[i] = 0.0;
    for (int64_t v = b * kPotThreads + threadIdx.x; v < nm; v += (int64_t)gridDim.x * kPotThreads)
        wsum += potential_point<K>(counts, V, nm, v, m.c_norm, p, over, present);
    if (over)
        raise_flag(HPF_FLAG_OVERFLOW);
    if (w_part) {
        const double s = block_sum(wsum, scratch);
        if (threadIdx.x == 0)
            w_part[b] = s * p.rho0_dV;
    }
}

hpf_status_t launch_field_potential(uint64_t* counts, const MeshK& m, int K, const PotK& p,
                                    float* V, double* w_part, uint8_t* present, hipStream_t s)
{
    int64_t nb = (m.nm + kPotThreads - 1) / kPotThreads;
    const int64_t cap = w_part ? HPF_NPART : 8192;
    if (nb > cap)
        nb = cap;
    auto* c = reinterpret_cast<unsigned long long*>(counts);
    const dim3 g((unsigned)nb), bl(kPotThreads);
    switch (K) {
    case 1: hipLaunchKernelGGL(k_field_potential<1>, g, bl, 0, s, c, m, p, V, w_part, present); break;
    case 2: hipLaunchKernelGGL(k_field_potential<2>, g, bl, 0, s, c, m, p, V, w_part, present); break;
    case 3: hipLaunchKernelGGL(k_field_potential<3>, g, bl, 0, s, c, m, p, V, w_part, present); break;
    case 4: hipLaunchKernelGGL(k_field_potential<4>, g, bl, 0, s, c, m, p, V, w_part, present); break;
    case 5: hipLaunchKernelGGL(k_field_potential<5>, g, bl, 0, s, c, m, p, V, w_part, present); break;
    case 6: hipLaunchKernelGGL(k_field_potential<6>, g, bl, 0, s, c, m, p, V, w_part, present); break;
    case 7: hipLaunchKernelGGL(k_field_potential<7>, g, bl, 0, s, c, m, p, V, w_part, present); break;
    case 8: hipLaunchKernelGGL(k_field_potential<8>, g, bl, 0, s, c, m, p, V, w_part, present); break;
    default: return HPF_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

// The density finish fused with the potential: for each brick of points (a
// persistent brick walk), the partial deposit boxes covering a point are
// summed (as in the cell scatter's sum pass) and added to the counts already
// held there (the beads that left their box), the counts are cleared, and V
// and the field-energy term follow as in k_field_potential. V and the counts
// it starts from are bitwise those of the finish + potential pair.
constexpr int kFPThreads = 256;

// One brick of the fused finish + potential: all threads of the workgroup
// call it; it begins with a barrier (the previous brick's cover lists may
// still be read) and returns this thread's field-energy terms.
template <int K>
__device__ __forceinline__ double finish_potential_brick(Cover (&cov)[3][kTcMaxB],
                                                         const unsigned long long* __restrict__ partials,
                                                         const TileK& tk, const PotK& p,
                                                         unsigned long long* __restrict__ counts,
                                                         float* __restrict__ V, int64_t brick, bool& over,
                                                         uint8_t* __restrict__ present)
{
    const MeshK& m = tk.m;
    const int64_t nm = m.nm;
    const int B = tk.B, P = tk.P, P3 = P * P * P;
    const int Mx = m.M[0], My = m.M[1];
    const int bxyz[3] = {(int)(brick % tk.nb[0]), (int)((brick / tk.nb[0]) % tk.nb[1]),
                         (int)(brick / ((int64_t)tk.nb[0] * tk.nb[1]))};
    int o[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        o[d] = min(B, m.M[d] - bxyz[d] * B);
    __syncthreads();
    brick_covers(cov, tk, K, bxyz, o);
    const int npts = o[0] * o[1] * o[2];
    double wsum = 0.0;
    for (int e = threadIdx.x; e < npts; e += (int)blockDim.x) {
        int ix, iy, iz;
        brick_point(e, o, B, ix, iy, iz);
        const Cover& cx = cov[0][ix];
        const Cover& cy = cov[1][iy];
        const Cover& cz = cov[2][iz];
        const int64_t dst = ((int64_t)(bxyz[2] * B + iz) * My + (bxyz[1] * B + iy)) * Mx + bxyz[0] * B + ix;
        unsigned long long n[K];
        bool held = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            n[k] = counts[(int64_t)k * nm + dst];
            held |= n[k] != 0ull;
        }
        if (cover2_ok(cx, cy, cz)) {
            const Cover2 c2 = cover2(cx, cy, cz);
#pragma unroll
            for (int k = 0; k < K; ++k)
                n[k] += cover2_sum(partials, c2, (int64_t)k * P3);
        } else {
            for (int a = 0; a < cz.n; ++a)
                for (int b2 = 0; b2 < cy.n; ++b2)
                    for (int c = 0; c < cx.n; ++c) {
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            n[k] += partials[cz.off[a] + cy.off[b2] + cx.off[c] + (int64_t)k * P3];
                    }
        }
        // the counts are cleared where they held anything (the few points that beads
        // outside their boxes reached); the others are zero already
        if (held)
#pragma unroll
            for (int k = 0; k < K; ++k)
                counts[(int64_t)k * nm + dst] = 0ull;
        if (present)
            present[dst] = composition<K>(n);
        wsum += potential_values<K>(n, V, nm, dst, m.c_norm, p, over);
    }
    return wsum;
}

template <int K>
__global__ __launch_bounds__(kFPThreads) void k_finish_potential(const unsigned long long* __restrict__ partials,
                                                                 TileK tk, PotK p,
                                                                 unsigned long long* __restrict__ counts,
                                                                 float* __restrict__ V, double* __restrict__ w_part,
                                                                 uint8_t* __restrict__ present)
{
    __shared__ Cover cov[3][kTcMaxB];
    __shared__ double scratch[kFPThreads / kWave];
    if (w_part)                                    // slots beyond this grid read as zero
        for (int64_t i = (int64_t)gridDim.x + blockIdx.x + (int64_t)threadIdx.x * gridDim.x; i < HPF_NPART;
             i += (int64_t)kFPThreads * gridDim.x)
            w_part[i] = 0.0;
    const BrickWalk w = brick_walk(tk.ntiles);
    double wsum = 0.0;
    bool over = false;
    for (int64_t brick = w.first; brick < w.end; brick += w.stride)
        wsum += finish_potential_brick<K>(cov, partials, tk, p, counts, V, brick, over, present);
    if (over)
        raise_flag(HPF_FLAG_OVERFLOW);
    if (w_part) {
        const double s = block_sum(wsum, scratch);
        if (threadIdx.x == 0)
            w_part[blockIdx.x] = s * p.rho0_dV;
    }
}

template <int K>
static hpf_status_t launch_finish_potential_k(const unsigned long long* partials, const TileK& tk, const PotK& p,
                                              unsigned long long* counts, float* V, double* w_part,
                                              uint8_t* present, hipStream_t s)
{
    // one brick per workgroup where the partial slots allow it (the dispatcher then
    // balances uneven bricks), else bricks walked by HPF_NPART workgroups
    const int64_t nb = std::min<int64_t>(tk.ntiles, HPF_NPART);
    hipLaunchKernelGGL(k_finish_potential<K>, dim3((unsigned)nb), dim3(kFPThreads), 0, s, partials, tk, p, counts, V,
                       w_part, present);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t launch_finish_potential(const unsigned long long* partials, const TileK& tk, int K, const PotK& p,
                                     uint64_t* counts, float* V, double* w_part, uint8_t* present, hipStream_t s)
{
    auto* c = reinterpret_cast<unsigned long long*>(counts);
    switch (K) {
    case 1: return launch_finish_potential_k<1>(partials, tk, p, c, V, w_part, present, s);
    case 2: return launch_finish_potential_k<2>(partials, tk, p, c, V, w_part, present, s);
    case 3: return launch_finish_potential_k<3>(partials, tk, p, c, V, w_part, present, s);
    case 4: return launch_finish_potential_k<4>(partials, tk, p, c, V, w_part, present, s);
    case 5: return launch_finish_potential_k<5>(partials, tk, p, c, V, w_part, present, s);
    case 6: return launch_finish_potential_k<6>(partials, tk, p, c, V, w_part, present, s);
    case 7: return launch_finish_potential_k<7>(partials, tk, p, c, V, w_part, present, s);
    case 8: return launch_finish_potential_k<8>(partials, tk, p, c, V, w_part, present, s);
    default: return HPF_EINVAL;
    }
}

constexpr int kGradX = 64, kGradY = 4;

// Centred gradient at mesh point (x, y, z): G = (gx, gy, gz) for the species whose
// bit is set in `listed` (the point's composition list; all species with ~0). Entries of
// species left out keep their previous values: a bead reads G of its own species only at
// the corners that its weights reach, all of which hold a non-zero count of its species.
__device__ __forceinline__ void gradient_point(const float* __restrict__ V, const MeshK& m, int K, int x, int y,
                                               int z, float3* __restrict__ G, uint32_t listed = ~0u)
{
    const int Mx = m.M[0], My = m.M[1], Mz = m.M[2];
    const int xp = next_wrap(x, Mx), xm = prev_wrap(x, Mx);
    const int64_t row = ((int64_t)z * My + y) * Mx;
    const int64_t rowyp = ((int64_t)z * My + next_wrap(y, My)) * Mx;
    const int64_t rowym = ((int64_t)z * My + prev_wrap(y, My)) * Mx;
    const int64_t rowzp = ((int64_t)next_wrap(z, Mz) * My + y) * Mx;
    const int64_t rowzm = ((int64_t)prev_wrap(z, Mz) * My + y) * Mx;
    const float hx = 0.5f * m.s[0], hy = 0.5f * m.s[1], hz = 0.5f * m.s[2];
    for (int k = 0; k < K; ++k) {
        if (!((listed >> k) & 1u))
            continue;
        const float* Vk = V + k * m.nm;
        float3 g;
        g.x = (Vk[row + xp] - Vk[row + xm]) * hx;
        g.y = (Vk[rowyp + x] - Vk[rowym + x]) * hy;
        g.z = (Vk[rowzp + x] - Vk[rowzm + x]) * hz;
        G[k * m.nm + row + x] = g;
    }
}

// One thread per mesh point: a 64 x 4 block covers a patch of an xy plane,
// so the +-x neighbours are in the same or adjacent cache lines and the +-y
// and +-z rows are re-read from L2 by neighbouring blocks. With `xcd` the
// blocks of one XCD take one contiguous run of patches (x, then y, then z), so
// those neighbours are in its own L2; without it consecutive patches go to
// different XCDs and meet in the Infinity Cache, which measured faster once
// the potential exceeds it (a 256^3 mesh of 3 species: 207 against 240 us; a
// 128^3 mesh of 2 species: 16.9 against 15.7 us with the contiguous runs).
constexpr int64_t kGradXcdBytes = int64_t(64) << 20;

__global__ __launch_bounds__(kGradX * kGradY) void k_field_gradient(const float* __restrict__ V,
                                                                    MeshK m, int K, int ntx, int nty,
                                                                    int xcd, float3* __restrict__ G,
                                                                    const uint8_t* __restrict__ present)
{
    const int64_t b = xcd ? xcd_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int tx = (int)(b % ntx), ty = (int)((b / ntx) % nty), z = (int)(b / ((int64_t)ntx * nty));
    const int x = tx * kGradX + threadIdx.x;
    const int y = ty * kGradY + threadIdx.y;
    if (x >= m.M[0] || y >= m.M[1])
        return;
    const uint32_t listed = present ? present[((int64_t)z * m.M[1] + y) * m.M[0] + x] : ~0u;
    gradient_point(V, m, K, x, y, z, G, listed);
}

hpf_status_t launch_field_gradient(const float* V, const MeshK& m, int K, float* G, const uint8_t* present,
                                   hipStream_t s)
{
    const int ntx = (m.M[0] + kGradX - 1) / kGradX, nty = (m.M[1] + kGradY - 1) / kGradY;
    const int64_t nb = (int64_t)ntx * nty * m.M[2];
    const int xcd = (int64_t)K * m.nm * 4 <= kGradXcdBytes ? 1 : 0;
    hipLaunchKernelGGL(k_field_gradient, dim3((unsigned)nb), dim3(kGradX, kGradY), 0, s, V, m, K, ntx, nty, xcd,
                       reinterpret_cast<float3*>(G), present);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

}  // namespace hpf
