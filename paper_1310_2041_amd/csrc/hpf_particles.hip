// Per-bead kernels: force interpolation from the gradient mesh (eq. 6,
// Algorithm 1 Kernel 4), harmonic bonds (eq. 7), the two half steps of
// velocity Verlet, and a fused kernel that runs all of them in one pass.
//
// One thread per bead; each workgroup walks a contiguous range of beads, and
// ranges are laid out so that consecutive ranges run on the same XCD
// (cell-sorted beads then share that XCD's L2 for mesh and partner reads).
// The separate kernels and the fused one call the same device functions in
// the same order, so they produce bitwise identical results.
#include <algorithm>

#include "hpf_common.hpp"
#include "hpf_thermo.hpp"

namespace hpf {

constexpr int kPThreads = 256;

// Work split of a per-bead kernel. The beads are cut into 8 contiguous
// ranges, one per XCD (workgroup b runs on XCD b % 8). Inside its range an
// XCD's workgroups take 256-bead chunks in turn (chunk c goes to the XCD's
// workgroup c mod n), so the chunks in flight at any moment are neighbours:
// with cell-sorted beads the gradient mesh and bond partners they touch form
// a compact window that stays in that XCD's L2 while it sweeps the range.
// The partial-sum slot of a workgroup is its launch index.
struct BeadWalk {
    int64_t begin, end;      // this XCD's range
    int64_t first, stride;   // first chunk start and chunk stride of this workgroup
    int64_t block;
};

__device__ __forceinline__ BeadWalk bead_walk(int64_t N, int64_t chunk = kPThreads)
{
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t ng = nb < 8 ? nb : 8;             // groups = XCDs that received workgroups
    const int64_t g = b % ng, idx = b / ng;
    const int64_t per_group = nb / ng + (g < nb % ng ? 1 : 0);
    const int64_t nchunk = (N + chunk - 1) / chunk;
    const int64_t c0 = nchunk * g / ng, c1 = nchunk * (g + 1) / ng;
    BeadWalk w;
    w.begin = min(N, c0 * chunk);
    w.end = min(N, c1 * chunk);
    w.first = w.begin + idx * chunk;
    w.stride = per_group * chunk;
    w.block = b;
    return w;
}

#define FOR_BEADS(w, i)                                                                   \
    for (int64_t _c = (w).first; _c < (w).end; _c += (w).stride)                          \
        for (int64_t i = _c + threadIdx.x; i < min(_c + (int64_t)kPThreads, (w).end); i += kPThreads)

// Partial-sum slots beyond the launched grid are cleared (slot s by block
// s mod grid), so a reduction over all HPF_NPART slots sees only this
// launch's sums.
__device__ __forceinline__ void clear_unused_slots(double* part, int rows)
{
    if (!part)
        return;
    for (int r = 0; r < rows; ++r)
        for (int64_t i = (int64_t)gridDim.x + blockIdx.x + (int64_t)threadIdx.x * gridDim.x; i < HPF_NPART;
             i += (int64_t)blockDim.x * gridDim.x)
            part[r * HPF_NPART + i] = 0.0;
}

struct BoxK {
    float L[3];
    float halfL[3];
};

// ------------------------------------------------------- device functions --

// Trilinear interpolation of the gradient at a bead from the 8 corner values
// g[a], a = x + 2y + 4z, with the exact FP32 dyadic 1-D weights (separable
// form of -sum_a (W_a / 2^48) G(c + a)).
__device__ __forceinline__ float3 interp8(const BeadCell& b, const float3 (&g)[8])
{
    const float ax1 = (float)b.q[0] * kInvOne, ax0 = (float)(kOne - b.q[0]) * kInvOne;
    const float ay1 = (float)b.q[1] * kInvOne, ay0 = (float)(kOne - b.q[1]) * kInvOne;
    const float az1 = (float)b.q[2] * kInvOne, az0 = (float)(kOne - b.q[2]) * kInvOne;
    float3 e00, e10, e01, e11, f0, f1, f;
    e00.x = ax0 * g[0].x + ax1 * g[1].x;
    e00.y = ax0 * g[0].y + ax1 * g[1].y;
    e00.z = ax0 * g[0].z + ax1 * g[1].z;
    e10.x = ax0 * g[2].x + ax1 * g[3].x;
    e10.y = ax0 * g[2].y + ax1 * g[3].y;
    e10.z = ax0 * g[2].z + ax1 * g[3].z;
    e01.x = ax0 * g[4].x + ax1 * g[5].x;
    e01.y = ax0 * g[4].y + ax1 * g[5].y;
    e01.z = ax0 * g[4].z + ax1 * g[5].z;
    e11.x = ax0 * g[6].x + ax1 * g[7].x;
    e11.y = ax0 * g[6].y + ax1 * g[7].y;
    e11.z = ax0 * g[6].z + ax1 * g[7].z;
    f0.x = ay0 * e00.x + ay1 * e10.x;
    f0.y = ay0 * e00.y + ay1 * e10.y;
    f0.z = ay0 * e00.z + ay1 * e10.z;
    f1.x = ay0 * e01.x + ay1 * e11.x;
    f1.y = ay0 * e01.y + ay1 * e11.y;
    f1.z = ay0 * e01.z + ay1 * e11.z;
    f.x = -(az0 * f0.x + az1 * f1.x);
    f.y = -(az0 * f0.y + az1 * f1.y);
    f.z = -(az0 * f0.z + az1 * f1.z);
    return f;
}

// The 8 corner values of cell b from species t's gradient mesh in memory.
__device__ __forceinline__ void corners_global(const BeadCell& b, int t, const MeshK& m,
                                               const float3* __restrict__ G, float3 (&g)[8])
{
    const float3* Gk = G + t * m.nm;
    const int32_t Mx = m.M[0], My = m.M[1], Mz = m.M[2];
    const int32_t x0 = b.c[0], x1 = next_wrap(x0, Mx);
    const int32_t y0 = b.c[1], y1 = next_wrap(y0, My);
    const int32_t z0 = b.c[2], z1 = next_wrap(z0, Mz);
    const int64_t r00 = ((int64_t)z0 * My + y0) * Mx, r10 = ((int64_t)z0 * My + y1) * Mx;
    const int64_t r01 = ((int64_t)z1 * My + y0) * Mx, r11 = ((int64_t)z1 * My + y1) * Mx;
    g[0] = Gk[r00 + x0];
    g[1] = Gk[r00 + x1];
    g[2] = Gk[r10 + x0];
    g[3] = Gk[r10 + x1];
    g[4] = Gk[r01 + x0];
    g[5] = Gk[r01 + x1];
    g[6] = Gk[r11 + x0];
    g[7] = Gk[r11 + x1];
}

// corners_global with 32-bit offsets into one buffer resource over the gradient mesh
// (at most kBufMeshBytes, which the launches check): the offsets need no 64-bit address
// arithmetic and keep fewer registers live while the loads are in flight.
constexpr int64_t kBufMeshBytes = 0x7fffffff;

__device__ __forceinline__ void corners_buffer(const BeadCell& b, int t, const MeshK& m,
                                               const float3* __restrict__ G, float3 (&g)[8])
{
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float3*>(G), 0, (int)kBufMeshBytes, 0x00020000);
    const uint32_t Mx = m.M[0], My = m.M[1];
    const uint32_t x0 = b.c[0], x1 = next_wrap(b.c[0], m.M[0]);
    const uint32_t y0 = b.c[1], y1 = next_wrap(b.c[1], m.M[1]);
    const uint32_t z0 = b.c[2], z1 = next_wrap(b.c[2], m.M[2]);
    const uint32_t tb = (uint32_t)t * (uint32_t)m.nm;
    const uint32_t r00 = tb + (z0 * My + y0) * Mx, r10 = tb + (z0 * My + y1) * Mx;
    const uint32_t r01 = tb + (z1 * My + y0) * Mx, r11 = tb + (z1 * My + y1) * Mx;
    const uint32_t off[8] = {r00 + x0, r00 + x1, r10 + x0, r10 + x1, r01 + x0, r01 + x1, r11 + x0, r11 + x1};
    typedef float v3f __attribute__((ext_vector_type(3)));
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const v3f v = __builtin_amdgcn_raw_buffer_load_b96(rs, (int)(off[a] * 12u), 0, 0);
        g[a] = make_float3(v.x, v.y, v.z);
    }
}

// Field force on one bead (eq. 6). False (and zero force) for a bead that
// cannot be binned or has a type >= K.
__device__ __forceinline__ bool field_force(const float3& r, int t, const MeshK& m, int K,
                                            const float3* __restrict__ G, float3& f)
{
    BeadCell b;
    f = make_float3(0.0f, 0.0f, 0.0f);
    if (!(bead_cell(r, m, b) && t < K))
        return false;
    float3 g[8];
    corners_global(b, t, m, G, g);
    f = interp8(b, g);
    return true;
}

// Field force on one bead read paper-literally from Algorithm 1 Kernels 3-4:
// along each axis the nearest vertex n (the cell's lower vertex when the
// quantised fraction is below one half, else the upper one) and the offset
// delta = u - n in [-1/2, 1/2); the backward difference V(n) - V(n - e) and the
// forward difference V(n + e) - V(n) are blended with the fraction ratios
// 1/2 - delta and 1/2 + delta (exact FP32 dyadics) and scaled by 1/h = s. V is
// the potential of the bead's own species, so the chi sum of Kernel 4 is
// already in it (eq. 6 is linear). False (and zero force) for a bead that
// cannot be binned or has a type >= K.
__device__ __forceinline__ bool field_force_staggered(const float3& r, int t, const MeshK& m, int K,
                                                      const float* __restrict__ V, float3& f)
{
    BeadCell b;
    f = make_float3(0.0f, 0.0f, 0.0f);
    if (!(bead_cell(r, m, b) && t < K))
        return false;
    const float* Vk = V + t * m.nm;
    int32_t n[3];
    float xf1[3], xf2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int32_t half = (int32_t)(kOne / 2);
        int32_t dq = (int32_t)b.q[d];
        n[d] = b.c[d];
        if (dq >= half) {
            n[d] = next_wrap(b.c[d], m.M[d]);
            dq -= (int32_t)kOne;
        }
        xf1[d] = (float)(half - dq) * kInvOne;
        xf2[d] = (float)(half + dq) * kInvOne;
    }
    const int32_t Mx = m.M[0], My = m.M[1], Mz = m.M[2];
    const int64_t row = ((int64_t)n[2] * My + n[1]) * Mx;
    const float v0 = Vk[row + n[0]];
    const float vxm = Vk[row + prev_wrap(n[0], Mx)], vxp = Vk[row + next_wrap(n[0], Mx)];
    const float vym = Vk[((int64_t)n[2] * My + prev_wrap(n[1], My)) * Mx + n[0]];
    const float vyp = Vk[((int64_t)n[2] * My + next_wrap(n[1], My)) * Mx + n[0]];
    const float vzm = Vk[((int64_t)prev_wrap(n[2], Mz) * My + n[1]) * Mx + n[0]];
    const float vzp = Vk[((int64_t)next_wrap(n[2], Mz) * My + n[1]) * Mx + n[0]];
    f.x = -(xf1[0] * (v0 - vxm) + xf2[0] * (vxp - v0)) * m.s[0];
    f.y = -(xf1[1] * (v0 - vym) + xf2[1] * (vyp - v0)) * m.s[1];
    f.z = -(xf1[2] * (v0 - vzm) + xf2[2] * (vzp - v0)) * m.s[2];
    return true;
}

// Sum of the harmonic bond forces on bead i over its table row, and its
// bond energy k (r - r0)^2 summed over its bonds (FP32).
template <bool kR0Zero>
__device__ __forceinline__ float3 bond_sum(int64_t i, const float3& xi, const float3* __restrict__ R,
                                           int64_t N, const int32_t* __restrict__ bonds, int D, float k,
                                           float r0, const BoxK& box, float& ei, bool& bad)
{
    const float two_k = 2.0f * k;
    float3 f = make_float3(0.0f, 0.0f, 0.0f);
    ei = 0.0f;
    for (int b = 0; b < D; ++b) {
        const int32_t j = bonds[(int64_t)b * N + i];
        if (j < 0)
            continue;
        if (j >= N) {
            bad = true;
            continue;
        }
        const float3 xj = R[j];
        const float dx = min_image(xj.x, xi.x, box.L[0], box.halfL[0]);
        const float dy = min_image(xj.y, xi.y, box.L[1], box.halfL[1]);
        const float dz = min_image(xj.z, xi.z, box.L[2], box.halfL[2]);
        const float r2 = dx * dx + dy * dy + dz * dz;
        float coef;
        if (kR0Zero) {
            coef = two_k;
            ei += k * r2;
        } else {
            const float r = sqrtf(r2);
            const float dr = r - r0;
            coef = r > 0.0f ? two_k * dr / r : 0.0f;
            ei += k * dr * dr;
        }
        f.x += coef * dx;
        f.y += coef * dy;
        f.z += coef * dz;
    }
    return f;
}

__device__ __forceinline__ void kick(float3& v, const float3& f, float im, float hdt)
{
    v.x += hdt * (f.x * im);
    v.y += hdt * (f.y * im);
    v.z += hdt * (f.z * im);
}

__device__ __forceinline__ void drift(float3& r, const float3& v, float dt, const BoxK& box)
{
    r.x = wrap_coord(r.x + dt * v.x, box.L[0]);
    r.y = wrap_coord(r.y + dt * v.y, box.L[1]);
    r.z = wrap_coord(r.z + dt * v.z, box.L[2]);
}

__device__ __forceinline__ bool finite3(const float3& a)
{
    return isfinite(a.x) && isfinite(a.y) && isfinite(a.z);
}

struct KinAcc {
    double ke = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    __device__ __forceinline__ void add(const float3& v, float im)
    {
        // beads of unit mass (every bead when no masses are given) skip the FP64 division
        double mass = 1.0;
        if (im != 1.0f)
            mass = 1.0 / (double)im;
        const double vx = v.x, vy = v.y, vz = v.z;
        ke += 0.5 * mass * (vx * vx + vy * vy + vz * vz);
        px += mass * vx;
        py += mass * vy;
        pz += mass * vz;
    }
    // rows of `stride` slots: KE, Px, Py, Pz
    __device__ __forceinline__ void store_rows(double* part, int64_t stride, int64_t slot, double* scratch)
    {
        const double a = block_sum(ke, scratch);
        const double b = block_sum(px, scratch);
        const double c = block_sum(py, scratch);
        const double d = block_sum(pz, scratch);
        if (threadIdx.x == 0) {
            part[0 * stride + slot] = a;
            part[1 * stride + slot] = b;
            part[2 * stride + slot] = c;
            part[3 * stride + slot] = d;
        }
    }
    __device__ __forceinline__ void store(double* part, int64_t slot, double* scratch)
    {
        store_rows(part, HPF_NPART, slot, scratch);
    }
};

// ---------------------------------------------------------------- kernels --

__global__ __launch_bounds__(kPThreads) void k_force_gather(const float3* __restrict__ R,
                                                            const uint8_t* __restrict__ T,
                                                            int64_t N, MeshK m, int K,
                                                            const float3* __restrict__ G,
                                                            float3* __restrict__ F)
{
    const BeadWalk w = bead_walk(N);
    bool bad = false;
    FOR_BEADS(w, i) {
        float3 f;
        bad |= !field_force(R[i], T[i], m, K, G, f);
        F[i] = make_float3(f.x, f.y, f.z);
    }
    if (bad)
        raise_flag(HPF_FLAG_BAD_BEAD);
}

__global__ __launch_bounds__(kPThreads) void k_force_gather_staggered(const float3* __restrict__ R,
                                                                      const uint8_t* __restrict__ T, int64_t N,
                                                                      MeshK m, int K, const float* __restrict__ V,
                                                                      float3* __restrict__ F)
{
    const BeadWalk w = bead_walk(N);
    bool bad = false;
    FOR_BEADS(w, i) {
        float3 f;
        bad |= !field_force_staggered(R[i], T[i], m, K, V, f);
        F[i] = make_float3(f.x, f.y, f.z);
    }
    if (bad)
        raise_flag(HPF_FLAG_BAD_BEAD);
}

// Angle parameters by type: U = k (theta - theta0)^2 (form 0) or
// k (cos theta - cos theta0)^2 (form 1), Bonded forces section.
struct AngleK {
    int ntypes;
    float k[8];
    float theta0[8];
    float cos0[8];
    int form[8];
};

// Force on bead i from its angle-table rows (each angle is evaluated by each of
// its three members, as the bonds are from both ends) and its share of their
// energy (one third each). theta is the angle at the middle bead between the
// minimum-image arms a = x_end1 - x_mid and b = x_end2 - x_mid;
// theta = atan2(|a x b|, a.b); dcos/dx_end1 = (b^ - c a^) / |a|,
// dcos/dx_end2 = (a^ - c b^) / |b|, dcos/dx_mid = -(their sum). For the harmonic
// form dU/dcos = -2k (theta - theta0) / sin(theta), sin(theta) floored at 1e-3.
__device__ __forceinline__ float3 angle_sum(int64_t i, const float3& xi, const float3* __restrict__ R, int64_t N,
                                            const int32_t* __restrict__ angles, int A, const AngleK& ak,
                                            const BoxK& box, double& ei, bool& bad)
{
    float3 f = make_float3(0.0f, 0.0f, 0.0f);
    for (int r = 0; r < A; ++r) {
        const int32_t p = angles[(3 * (int64_t)r + 0) * N + i];
        const int32_t q = angles[(3 * (int64_t)r + 1) * N + i];
        const int32_t code = angles[(3 * (int64_t)r + 2) * N + i];
        if (p < 0)
            continue;
        const int role = code & 1, type = code >> 1;
        if (p >= N || q < 0 || q >= N || type >= ak.ntypes) {
            bad = true;
            continue;
        }
        const float3 xp = R[p], xq = R[q];
        // the middle bead and the two ends
        const float3 xm = role ? xi : xp;
        const float3 x1 = role ? xp : xi;
        float a[3], b[3];
        a[0] = min_image(x1.x, xm.x, box.L[0], box.halfL[0]);
        a[1] = min_image(x1.y, xm.y, box.L[1], box.halfL[1]);
        a[2] = min_image(x1.z, xm.z, box.L[2], box.halfL[2]);
        b[0] = min_image(xq.x, xm.x, box.L[0], box.halfL[0]);
        b[1] = min_image(xq.y, xm.y, box.L[1], box.halfL[1]);
        b[2] = min_image(xq.z, xm.z, box.L[2], box.halfL[2]);
        const float na = sqrtf(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        const float nb = sqrtf(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        const float dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
        const float cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
        const float cr = sqrtf(cx * cx + cy * cy + cz * cz);
        const float c = dot / (na * nb);
        float U, dUdc;
        if (ak.form[type] == 0) {
            const float th = atan2f(cr, dot) - ak.theta0[type];
            const float st = fmaxf(cr / (na * nb), 1e-3f);
            U = ak.k[type] * th * th;
            dUdc = -2.0f * ak.k[type] * th / st;
        } else {
            const float dc = c - ak.cos0[type];
            U = ak.k[type] * dc * dc;
            dUdc = 2.0f * ak.k[type] * dc;
        }
        float g[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float g1 = (b[d] / nb - c * a[d] / na) / na;
            const float g2 = (a[d] / na - c * b[d] / nb) / nb;
            g[d] = role ? -(g1 + g2) : g1;
        }
        f.x -= dUdc * g[0];
        f.y -= dUdc * g[1];
        f.z -= dUdc * g[2];
        ei += (double)U / 3.0;
    }
    return f;
}

// F_i += the angle forces on bead i; optional FP64 energy partials.
__global__ __launch_bounds__(kPThreads) void k_angle_forces(const float3* __restrict__ R, int64_t N,
                                                            const int32_t* __restrict__ angles, int A, AngleK ak,
                                                            BoxK box, float3* __restrict__ F,
                                                            double* __restrict__ e_part)
{
    __shared__ double scratch[kPThreads / kWave];
    const BeadWalk w = bead_walk(N);
    clear_unused_slots(e_part, 1);
    double e = 0.0;
    bool bad = false;
    FOR_BEADS(w, i) {
        const float3 fa = angle_sum(i, R[i], R, N, angles, A, ak, box, e, bad);
        float3 f = F[i];
        f.x += fa.x;
        f.y += fa.y;
        f.z += fa.z;
        F[i] = f;
    }
    if (bad)
        raise_flag(HPF_FLAG_BAD_BOND);
    if (e_part) {
        const double s = block_sum(e, scratch);
        if (threadIdx.x == 0)
            e_part[w.block] = s;
    }
}

// F_i += sum_j 2k (r - r0) d / r over the bead's own table row; E partials
// accumulate k (r - r0)^2 / 2 per bond end (each bond is seen from both ends).
template <bool kR0Zero>
__global__ __launch_bounds__(kPThreads) void k_bond_forces(const float3* __restrict__ R, int64_t N,
                                                           const int32_t* __restrict__ bonds, int D,
                                                           float k, float r0, BoxK box,
                                                           float3* __restrict__ F,
                                                           double* __restrict__ e_part)
{
    __shared__ double scratch[kPThreads / kWave];
    const BeadWalk w = bead_walk(N);
    clear_unused_slots(e_part, 1);
    double e = 0.0;
    bool bad = false;
    FOR_BEADS(w, i) {
        const float3 xi = R[i];
        float ei;
        const float3 fb = bond_sum<kR0Zero>(i, xi, R, N, bonds, D, k, r0, box, ei, bad);
        float3 f = F[i];
        f.x += fb.x;
        f.y += fb.y;
        f.z += fb.z;
        F[i] = f;
        e += 0.5 * (double)ei;
    }
    if (bad)
        raise_flag(HPF_FLAG_BAD_BOND);
    if (e_part) {
        const double s = block_sum(e, scratch);
        if (threadIdx.x == 0)
            e_part[w.block] = s;
    }
}

__global__ __launch_bounds__(kPThreads) void k_verlet_half1(float3* __restrict__ R,
                                                            float3* __restrict__ Vel,
                                                            const float3* __restrict__ F,
                                                            const float* __restrict__ inv_mass,
                                                            int64_t N, float dt, BoxK box)
{
    const BeadWalk w = bead_walk(N);
    const float hdt = 0.5f * dt;
    bool bad = false;
    FOR_BEADS(w, i) {
        const float im = inv_mass ? inv_mass[i] : 1.0f;
        float3 v = Vel[i];
        float3 r = R[i];
        kick(v, F[i], im, hdt);
        drift(r, v, dt, box);
        bad |= !(finite3(r) && finite3(v));
        Vel[i] = v;
        R[i] = r;
    }
    if (bad)
        raise_flag(HPF_FLAG_NONFINITE);
}

__global__ __launch_bounds__(kPThreads) void k_verlet_half2(float3* __restrict__ Vel,
                                                            const float3* __restrict__ F,
                                                            const float* __restrict__ inv_mass,
                                                            int64_t N, float dt,
                                                            double* __restrict__ kin_part)
{
    __shared__ double scratch[kPThreads / kWave];
    const BeadWalk w = bead_walk(N);
    clear_unused_slots(kin_part, 4);
    const float hdt = 0.5f * dt;
    KinAcc acc;
    bool bad = false;
    FOR_BEADS(w, i) {
        const float im = inv_mass ? inv_mass[i] : 1.0f;
        float3 v = Vel[i];
        kick(v, F[i], im, hdt);
        bad |= !finite3(v);
        Vel[i] = v;
        acc.add(v, im);
    }
    if (bad)
        raise_flag(HPF_FLAG_NONFINITE);
    if (kin_part)
        acc.store(kin_part, w.block, scratch);
}

// One bead of the fused pass: field force + bond forces at x_n, second half
// kick of step n (kinetic-energy partials at v_n), first half kick and drift
// of step n + 1, written to R_next. With kThermo the Andersen collisions of th act
// on v_n (a separate instantiation, so the NVE passes keep their register budget).
template <bool kR0Zero, bool kThermo>
__device__ __forceinline__ float3 advance_bead(int64_t i, const float3* __restrict__ R, float3* __restrict__ R_next,
                                             float3* __restrict__ Vel, const uint8_t* __restrict__ T,
                                             int64_t N, const MeshK& m, int K, const float3* __restrict__ G,
                                             const int32_t* __restrict__ bonds, int D, float k, float r0,
                                             const BoxK& box, const float* __restrict__ inv_mass, float dt,
                                             float hdt, float3* __restrict__ F_out, KinAcc& acc, double& e,
                                             bool& bad_bead, bool& bad_bond, bool& nonfinite,
                                             const ThermoK& th, uint64_t tstep)
{
    float3 r = R[i];
    float3 ff;
    bad_bead |= !field_force(r, T[i], m, K, G, ff);
    float ei;
    const float3 fb = bond_sum<kR0Zero>(i, r, R, N, bonds, D, k, r0, box, ei, bad_bond);
    float3 f = make_float3(ff.x, ff.y, ff.z);
    f.x += fb.x;
    f.y += fb.y;
    f.z += fb.z;
    e += 0.5 * (double)ei;
    if (F_out)
        F_out[i] = f;
    const float im = inv_mass ? inv_mass[i] : 1.0f;
    float3 v = Vel[i];
    kick(v, f, im, hdt);                 // v_n
    if (kThermo && th.thr)
        andersen_collide(th, tstep, th.tag[i], im, v);
    acc.add(v, im);
    kick(v, f, im, hdt);                 // v_{n+1/2}
    drift(r, v, dt, box);                // x_{n+1}
    nonfinite |= !(finite3(r) && finite3(v));
    Vel[i] = v;
    R_next[i] = r;
    return r;
}

// Software-pipelined form of advance_bead for bond tables of at most two rows.
// A bead's own data (position, velocity, type, bond row, inverse mass) is
// loaded one loop iteration ahead, and those loads are issued after the
// current bead's corner and partner loads: vector memory operations retire in
// issue order for the wait counter, so loads issued earlier would hold up the
// wait for the corners. The arithmetic is that of advance_bead, in the same
// order, so results are bitwise equal. When the pass streams its data from HBM (kNT), a
// wave issues its corner and partner loads at raised wave priority (s_setprio 1, back to
// 0 once they are out), so the arbiter lets it send them back to back rather than between
// other waves' arithmetic: the 10M-bead blend's depositing pass went from 257 to 248 us
// and the 100M-bead step from 4.27 to 4.21 ms; a system inside the Infinity Cache (1M
// beads) ran 4 us slower with it, and keeps the default priority.
constexpr int kPreBonds = 2;

struct BeadIn {
    float3 r, v;
    float im;
    int t;
    int32_t tag;
    int32_t j[kPreBonds];
};

template <bool kThermo, bool kNT>
__device__ __forceinline__ void bead_fetch(BeadIn& p, int64_t i, const float3* __restrict__ R,
                                           const float3* __restrict__ Vel, const uint8_t* __restrict__ T,
                                           const int32_t* __restrict__ bonds, int D, int64_t N,
                                           const float* __restrict__ inv_mass, const ThermoK& th)
{
    p.r = R[i];                       // also read as bond partners: cached
    p.v = load_hint<kNT>(Vel + i);
    p.t = load_hint<kNT>(T + i);
    p.im = inv_mass ? inv_mass[i] : 1.0f;
    p.tag = (kThermo && th.thr) ? th.tag[i] : 0;
#pragma unroll
    for (int b = 0; b < kPreBonds; ++b)
        p.j[b] = b < D ? load_hint<kNT>(bonds + (int64_t)b * N + i) : -1;
}

struct BeadLoads {
    float3 g[8];
    float3 xj[kPreBonds];
    BeadCell b;
    bool ok;
};

// Cell of the bead, its 8 corner loads (corners_buffer; a bead that cannot be binned
// loads the corners of cell 0 and gets no field force) and its partner loads (an index
// outside [0, N) loads the bead itself; the bond is then skipped or flagged).
__device__ __forceinline__ void bead_issue(BeadLoads& L, const BeadIn& p, int64_t i, const MeshK& m, int K,
                                           const float3* __restrict__ G, const float3* __restrict__ R, int64_t N)
{
    L.ok = bead_cell(p.r, m, L.b) && p.t < K;
    BeadCell c = L.b;
    if (!L.ok)
        c.c[0] = c.c[1] = c.c[2] = 0;
    corners_buffer(c, L.ok ? p.t : 0, m, G, L.g);
#pragma unroll
    for (int b = 0; b < kPreBonds; ++b) {
        const int32_t j = p.j[b];
        L.xj[b] = R[(j >= 0 && j < N) ? (int64_t)j : i];
    }
}

template <bool kR0Zero, bool kThermo, bool kNT>
__device__ __forceinline__ float3 bead_finish(int64_t i, const BeadIn& p, const BeadLoads& L,
                                              float3* __restrict__ R_next, float3* __restrict__ Vel, int64_t N,
                                              int D, float k, float r0, const BoxK& box, float dt, float hdt,
                                              float3* __restrict__ F_out, KinAcc& acc, double& e, bool& bad_bead,
                                              bool& bad_bond, bool& nonfinite, const ThermoK& th, uint64_t tstep)
{
    float3 r = p.r;
    float3 ff = make_float3(0.0f, 0.0f, 0.0f);
    if (L.ok)
        ff = interp8(L.b, L.g);
    bad_bead |= !L.ok;
    // bond forces: the operations of bond_sum
    const float two_k = 2.0f * k;
    float3 fb = make_float3(0.0f, 0.0f, 0.0f);
    float ei = 0.0f;
#pragma unroll
    for (int b = 0; b < kPreBonds; ++b) {
        if (b >= D)
            break;
        const int32_t j = p.j[b];
        if (j < 0)
            continue;
        if (j >= N) {
            bad_bond = true;
            continue;
        }
        const float3 xj = L.xj[b];
        const float dx = min_image(xj.x, r.x, box.L[0], box.halfL[0]);
        const float dy = min_image(xj.y, r.y, box.L[1], box.halfL[1]);
        const float dz = min_image(xj.z, r.z, box.L[2], box.halfL[2]);
        const float r2 = dx * dx + dy * dy + dz * dz;
        float coef;
        if (kR0Zero) {
            coef = two_k;
            ei += k * r2;
        } else {
            const float rr = sqrtf(r2);
            const float dr = rr - r0;
            coef = rr > 0.0f ? two_k * dr / rr : 0.0f;
            ei += k * dr * dr;
        }
        fb.x += coef * dx;
        fb.y += coef * dy;
        fb.z += coef * dz;
    }
    float3 f = make_float3(ff.x, ff.y, ff.z);
    f.x += fb.x;
    f.y += fb.y;
    f.z += fb.z;
    e += 0.5 * (double)ei;
    if (F_out)
        F_out[i] = f;
    float3 v = p.v;
    kick(v, f, p.im, hdt);               // v_n
    if (kThermo && th.thr)
        andersen_collide(th, tstep, p.tag, p.im, v);
    acc.add(v, p.im);
    kick(v, f, p.im, hdt);               // v_{n+1/2}
    drift(r, v, dt, box);                // x_{n+1}
    nonfinite |= !(finite3(r) && finite3(v));
    store_hint<kNT>(Vel + i, v);
    store_hint<kNT>(R_next + i, r);
    return r;
}

// Fused pass over the beads. Positions go to R_next so that bond partners
// are always read at x_n.
// The software-pipelined form runs 512-thread workgroups over 512-bead chunks
// (4% faster at 10M beads than 256); the general loop keeps kPThreads.
constexpr int kAdvPipeThreads = 512;

template <bool kR0Zero, bool kPipe, bool kThermo, bool kNT>
__global__ __launch_bounds__(kAdvPipeThreads) void k_advance(const float3* __restrict__ R,
                                                       float3* __restrict__ R_next,
                                                       float3* __restrict__ Vel,
                                                       const uint8_t* __restrict__ T, int64_t N,
                                                       MeshK m, int K, const float3* __restrict__ G,
                                                       const int32_t* __restrict__ bonds, int D,
                                                       float k, float r0, BoxK box,
                                                       const float* __restrict__ inv_mass, float dt,
                                                       float3* __restrict__ F_out,
                                                       double* __restrict__ e_part,
                                                       double* __restrict__ kin_part, ThermoK th)
{
    __shared__ double scratch[kAdvPipeThreads / kWave];
    const uint64_t tstep = thermo_step(th);
    const BeadWalk w = bead_walk(N, kPipe ? kAdvPipeThreads : kPThreads);
    clear_unused_slots(e_part, 1);
    clear_unused_slots(kin_part, 4);
    const float hdt = 0.5f * dt;
    KinAcc acc;
    double e = 0.0;
    bool bad_bead = false, bad_bond = false, nonfinite = false;
    if (kPipe) {
        // software-pipelined as in k_advance_scatter (bond table of at most kPreBonds
        // rows): a thread's beads are i, i + stride, ... (one per chunk of its walk), and
        // the next one's own loads stay in flight through this one's arithmetic
        int64_t i = w.first + threadIdx.x;
        BeadIn cur;
        if (i < w.end)
            bead_fetch<kThermo, kNT>(cur, i, R, Vel, T, bonds, D, N, inv_mass, th);
        for (; i < w.end; i += w.stride) {
            BeadLoads L;
            if constexpr (kNT)
                __builtin_amdgcn_s_setprio(1);
            bead_issue(L, cur, i, m, K, G, R, N);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (kNT)
                __builtin_amdgcn_s_setprio(0);
            BeadIn nxt;
            bead_fetch<kThermo, kNT>(nxt, i + w.stride < w.end ? i + w.stride : i, R, Vel, T, bonds, D, N, inv_mass,
                                th);
            __builtin_amdgcn_sched_barrier(0);
            bead_finish<kR0Zero, kThermo, kNT>(i, cur, L, R_next, Vel, N, D, k, r0, box, dt, hdt, F_out, acc, e,
                                          bad_bead, bad_bond, nonfinite, th, tstep);
            cur = nxt;
        }
    } else {
        FOR_BEADS(w, i) {
            advance_bead<kR0Zero, kThermo>(i, R, R_next, Vel, T, N, m, K, G, bonds, D, k, r0, box, inv_mass, dt,
                                           hdt, F_out, acc, e, bad_bead, bad_bond, nonfinite, th, tstep);
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
            e_part[w.block] = s;
    }
    if (kin_part)
        acc.store(kin_part, w.block, scratch);
}

// The fused pass plus the density deposit of the new positions, one brick of
// the last sort at a time (bricks walked as the beads are in bead_walk: one
// contiguous run of bricks per XCD, taken in turn by its workgroups). Each bead is
// advanced exactly as in k_advance; its new position x_{n+1} is deposited into
// the brick's LDS box (the deposit box of the cell scatter, P = B + 1 + 2h
// points per axis), which is stored to the brick's partial buffer when the
// brick is done. New positions outside the box, and every bead the sort could
// not bin, are added to `counts` with global atomics; the partial sum pass
// (k_scatter_sum<true>, or the fused finish + potential) then completes the
// counts of x_{n+1}.
// Workgroup size: 512 threads (two workgroups of 8 waves per CU at 4 waves
// per SIMD); with the software-pipelined loop this measured faster than 256
// threads at every mesh size tried, and a small mesh still fills the chip.
// kPipe selects the software-pipelined bead loop (bond tables of at most
// kPreBonds rows, gradient meshes of at most kBufMeshBytes); the plain loop serves
// the others. kNT puts the nontemporal hint on the pipelined loop's streamed data
// and on the stored deposit boxes.
constexpr int kASThreadsDefault = 512;
constexpr int kASThreadsWide = 768;

template <bool kR0Zero, int kASThreads, bool kPipe, bool kThermo, bool kNT>
// The second bound is waves per SIMD. The production form (512 threads, r0 = 0, no
// thermostat) keeps two workgroups per CU, 4 waves per SIMD (at most 128 VGPRs, which it
// fits without spilling); the others take 3 (at most 168), as does a 768-thread workgroup,
// which runs alone on its CU next to its large deposit box.
__global__ __launch_bounds__(kASThreads, kASThreads == kASThreadsDefault && kR0Zero && !kThermo ? 4 : 3) void
k_advance_scatter(
    const float3* __restrict__ R,
                                                                float3* __restrict__ R_next,
                                                                float3* __restrict__ Vel,
                                                                const uint8_t* __restrict__ T, int64_t N,
                                                                TileK tk, int K, const float3* __restrict__ G,
                                                                const int32_t* __restrict__ bonds, int D,
                                                                float k, float r0, BoxK box,
                                                                const float* __restrict__ inv_mass, float dt,
                                                                const uint32_t* __restrict__ cell_start,
                                                                unsigned long long* __restrict__ partials,
                                                                unsigned long long* __restrict__ counts,
                                                                float3* __restrict__ F_out,
                                                                double* __restrict__ e_part,
                                                                double* __restrict__ kin_part, ThermoK th)
{
    extern __shared__ unsigned long long dbox[];
    const uint64_t tstep = thermo_step(th);
    __shared__ double scratch[kASThreads / kWave];
    clear_unused_slots(e_part, 1);
    clear_unused_slots(kin_part, 4);
    const MeshK& m = tk.m;
    const int B = tk.B, P = tk.P, h = tk.h;
    const int P3 = P * P * P;
    const int nbox = K * P3;
    const BrickWalk w = brick_walk(tk.ntiles + 1);
    const float hdt = 0.5f * dt;
    KinAcc acc;
    double e = 0.0;
    bool bad_bead = false, bad_bond = false, nonfinite = false;
    for (int64_t item = w.first; item < w.end; item += w.stride) {
        if (item < tk.ntiles) {
            const int bx = (int)(item % tk.nb[0]);
            const int by = (int)((item / tk.nb[0]) % tk.nb[1]);
            const int bz = (int)(item / ((int64_t)tk.nb[0] * tk.nb[1]));
            const int x0 = bx * B, y0 = by * B, z0 = bz * B;
            const int ox = min(B, m.M[0] - x0), oy = min(B, m.M[1] - y0), oz = min(B, m.M[2] - z0);
            __syncthreads();                          // the previous brick's box is stored
            for (int q = threadIdx.x; q < nbox; q += kASThreads)
                dbox[q] = 0ull;
            __syncthreads();
            const int64_t first = cell_start[item];
            const int64_t last = min((int64_t)cell_start[item + 1], N);
            if (kPipe) {
                // Bond table of at most kPreBonds rows. The next bead's own loads go out
                // after this bead's corner and partner loads (the scheduling barriers keep
                // that order) and stay in flight through its arithmetic; a thread's last
                // bead fetches a valid bead again.
                int64_t i = first + threadIdx.x;
                BeadIn cur;
                if (i < last)
                    bead_fetch<kThermo, kNT>(cur, i, R, Vel, T, bonds, D, N, inv_mass, th);
                for (; i < last; i += kASThreads) {
                    BeadLoads L;
                    if constexpr (kNT)
                        __builtin_amdgcn_s_setprio(1);
                    bead_issue(L, cur, i, m, K, G, R, N);
                    __builtin_amdgcn_sched_barrier(0);
                    if constexpr (kNT)
                        __builtin_amdgcn_s_setprio(0);
                    BeadIn nxt;
                    bead_fetch<kThermo, kNT>(nxt, min(i + kASThreads, last - 1), R, Vel, T, bonds, D, N, inv_mass, th);
                    __builtin_amdgcn_sched_barrier(0);
                    const float3 rn = bead_finish<kR0Zero, kThermo, kNT>(i, cur, L, R_next, Vel, N, D, k, r0, box, dt, hdt,
                                                           F_out, acc, e, bad_bead, bad_bond, nonfinite, th,
                                                           tstep);
                    const int t = cur.t;
                    BeadCell b;
                    int lx, ly, lz;
                    if (bead_cell(rn, m, b) && t < K &&
                        brick_box_cell(b, m, x0, y0, z0, ox, oy, oz, h, lx, ly, lz))
                        box_deposit(dbox, P, t, lx, ly, lz, b);
                    else
                        bad_bead |= !deposit_global(rn, t, K, m, counts);
                    cur = nxt;
                }
            } else {
                for (int64_t i = first + threadIdx.x; i < last; i += kASThreads) {
                    const float3 rn = advance_bead<kR0Zero, kThermo>(i, R, R_next, Vel, T, N, m, K, G, bonds, D, k,
                                                            r0, box, inv_mass, dt, hdt, F_out, acc, e, bad_bead,
                                                            bad_bond, nonfinite, th, tstep);
                    const int t = T[i];
                    BeadCell b;
                    int lx, ly, lz;
                    if (bead_cell(rn, m, b) && t < K &&
                        brick_box_cell(b, m, x0, y0, z0, ox, oy, oz, h, lx, ly, lz))
                        box_deposit(dbox, P, t, lx, ly, lz, b);
                    else
                        bad_bead |= !deposit_global(rn, t, K, m, counts);
                }
            }
            __syncthreads();
            unsigned long long* out = partials + item * (int64_t)nbox;
            for (int q = threadIdx.x; q < nbox; q += kASThreads)
                store_hint<kNT>(out + q, dbox[q]);
        } else {
            const int64_t first = cell_start[tk.NK];
            for (int64_t i = first + threadIdx.x; i < N; i += kASThreads) {
                const float3 rn = advance_bead<kR0Zero, kThermo>(i, R, R_next, Vel, T, N, m, K, G, bonds, D, k, r0,
                                                        box, inv_mass, dt, hdt, F_out, acc, e, bad_bead, bad_bond,
                                                        nonfinite, th, tstep);
                bad_bead |= !deposit_global(rn, T[i], K, m, counts);
            }
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
            e_part[blockIdx.x] = s;
    }
    if (kin_part)
        acc.store(kin_part, blockIdx.x, scratch);
}

// ---------------------------------------------------------------- launches --

static int64_t bead_blocks(int64_t N, int64_t cap)
{
    int64_t nb = (N + kPThreads - 1) / kPThreads;
    if (nb > cap)
        nb = cap;
    return nb < 1 ? 1 : nb;
}

hpf_status_t launch_force_gather(const float* R, const uint8_t* T, int64_t N, const MeshK& m,
                                 int K, const float* G, float* F, hipStream_t s)
{
    if (N == 0)
        return HPF_OK;
    hipLaunchKernelGGL(k_force_gather, dim3((unsigned)bead_blocks(N, 1 << 20)), dim3(kPThreads),
                       0, s, reinterpret_cast<const float3*>(R), T, N, m, K,
                       reinterpret_cast<const float3*>(G), reinterpret_cast<float3*>(F));
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t launch_force_gather_staggered(const float* R, const uint8_t* T, int64_t N, const MeshK& m, int K,
                                           const float* V, float* F, hipStream_t s)
{
    if (N == 0)
        return HPF_OK;
    hipLaunchKernelGGL(k_force_gather_staggered, dim3((unsigned)bead_blocks(N, 1 << 20)), dim3(kPThreads), 0, s,
                       reinterpret_cast<const float3*>(R), T, N, m, K, V, reinterpret_cast<float3*>(F));
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t launch_angle_forces(const float* R, int64_t N, const int32_t* angles, int A, const AngleK& ak,
                                 const BoxK& box, float* F, double* e_part, hipStream_t s)
{
    if (N == 0 && !e_part)
        return HPF_OK;
    const int64_t nb = bead_blocks(N, e_part ? HPF_NPART : (1 << 20));
    hipLaunchKernelGGL(k_angle_forces, dim3((unsigned)nb), dim3(kPThreads), 0, s, reinterpret_cast<const float3*>(R),
                       N, angles, A, ak, box, reinterpret_cast<float3*>(F), e_part);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t launch_bond_forces(const float* R, int64_t N, const int32_t* bonds, int D, float k,
                                float r0, const BoxK& box, float* F, double* e_part, hipStream_t s)
{
    if (N == 0 && !e_part)
        return HPF_OK;
    const int64_t nb = bead_blocks(N, e_part ? HPF_NPART : (1 << 20));
    const dim3 g((unsigned)nb), bl(kPThreads);
    auto* Rp = reinterpret_cast<const float3*>(R);
    auto* Fp = reinterpret_cast<float3*>(F);
    if (r0 == 0.0f)
        hipLaunchKernelGGL(k_bond_forces<true>, g, bl, 0, s, Rp, N, bonds, D, k, r0, box, Fp, e_part);
    else
        hipLaunchKernelGGL(k_bond_forces<false>, g, bl, 0, s, Rp, N, bonds, D, k, r0, box, Fp, e_part);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t launch_verlet(float* R, float* Vel, const float* F, const float* inv_mass, int64_t N,
                           float dt, const BoxK& box, int half, double* kin_part, hipStream_t s)
{
    if (N == 0 && !(half == 2 && kin_part))
        return HPF_OK;
    auto* Rp = reinterpret_cast<float3*>(R);
    auto* Vp = reinterpret_cast<float3*>(Vel);
    auto* Fp = reinterpret_cast<const float3*>(F);
    if (half == 1) {
        hipLaunchKernelGGL(k_verlet_half1, dim3((unsigned)bead_blocks(N, 1 << 20)), dim3(kPThreads),
                           0, s, Rp, Vp, Fp, inv_mass, N, dt, box);
    } else {
        const int64_t nb = bead_blocks(N, kin_part ? HPF_NPART : (1 << 20));
        hipLaunchKernelGGL(k_verlet_half2, dim3((unsigned)nb), dim3(kPThreads), 0, s, Vp, Fp,
                           inv_mass, N, dt, kin_part);
    }
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

// Bytes one fused pass streams: bead rows read and written, the bond slots it
// prefetches, the gradient mesh and the stored deposit boxes.
static int64_t streamed_bytes(int64_t N, int D, int K, const MeshK& m, int64_t box_bytes)
{
    return N * (49 + 4 * (int64_t)std::min(D, kPreBonds)) + (int64_t)K * m.nm * 12 + box_bytes;
}

using AdvFn = void (*)(const float3*, float3*, float3*, const uint8_t*, int64_t, MeshK, int, const float3*,
                       const int32_t*, int, float, float, BoxK, const float*, float, float3*, double*, double*,
                       ThermoK);

template <bool kPipe, bool kNT>
static AdvFn advance_fn(bool thermo, bool r0z)
{
    return thermo ? (r0z ? k_advance<true, kPipe, true, kNT> : k_advance<false, kPipe, true, kNT>)
                  : (r0z ? k_advance<true, kPipe, false, kNT> : k_advance<false, kPipe, false, kNT>);
}

hpf_status_t launch_advance(const float* R, float* R_next, float* Vel, const uint8_t* T, int64_t N,
                            const MeshK& m, int K, const float* G, const int32_t* bonds, int D, float k,
                            float r0, const BoxK& box, const float* inv_mass, float dt, float* F_out,
                            double* e_part, double* kin_part, const ThermoK& th, hipStream_t s)
{
    if (N == 0 && !e_part && !kin_part)
        return HPF_OK;
    // the software-pipelined bead loop serves bond tables of up to kPreBonds rows and
    // gradient meshes of up to kBufMeshBytes
    const bool pipe = D <= kPreBonds && (int64_t)K * m.nm * 12 <= kBufMeshBytes;
    const int threads = pipe ? kAdvPipeThreads : kPThreads;
    const int64_t cap = (e_part || kin_part) ? HPF_NPART : (1 << 20);
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((N + threads - 1) / threads, cap));
    const dim3 g((unsigned)nb), bl(threads);
    auto* Rp = reinterpret_cast<const float3*>(R);
    auto* Rn = reinterpret_cast<float3*>(R_next);
    auto* Vp = reinterpret_cast<float3*>(Vel);
    auto* Gp = reinterpret_cast<const float3*>(G);
    auto* Fo = reinterpret_cast<float3*>(F_out);
    const bool thermo = th.thr != 0, r0z = r0 == 0.0f;
    const bool nt = pipe && streamed_bytes(N, D, K, m, 0) > kStreamHintBytes;
    const AdvFn fn = pipe ? (nt ? advance_fn<true, true>(thermo, r0z) : advance_fn<true, false>(thermo, r0z))
                          : advance_fn<false, false>(thermo, r0z);
    hipLaunchKernelGGL(fn, g, bl, 0, s, Rp, Rn, Vp, T, N, m, K, Gp, bonds, D, k, r0, box, inv_mass, dt, Fo,
                       e_part, kin_part, th);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

template <bool kR0Zero, int kThreads, bool kPipe, bool kThermo, bool kNT>
static hpf_status_t launch_advance_scatter_t(const float3* Rp, float3* Rn, float3* Vp, const uint8_t* T, int64_t N,
                                             const TileK& tk, int K, const float3* Gp, const int32_t* bonds, int D,
                                             float k, float r0, const BoxK& box, const float* inv_mass, float dt,
                                             const uint32_t* cell_start, unsigned long long* partials,
                                             unsigned long long* counts, float3* Fo, double* e_part,
                                             double* kin_part, const ThermoK& th, hipStream_t s)
{
    const size_t smem = sizeof(unsigned long long) * (size_t)K * tk.P * tk.P * tk.P;
    const void* fn = reinterpret_cast<const void*>(k_advance_scatter<kR0Zero, kThreads, kPipe, kThermo, kNT>);
    if (smem > 65536 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess)
        return HPF_EINVAL;
    // one brick per workgroup where the partial slots allow it, so the dispatcher balances
    // uneven bricks; larger meshes walk their bricks with HPF_NPART workgroups
    const int64_t nb = std::min<int64_t>(tk.ntiles + 1, HPF_NPART);
    const dim3 g((unsigned)nb), bl(kThreads);
    hipLaunchKernelGGL((k_advance_scatter<kR0Zero, kThreads, kPipe, kThermo, kNT>), g, bl, smem, s, Rp, Rn, Vp, T, N, tk,
                       K, Gp, bonds, D, k, r0, box, inv_mass, dt, cell_start, partials, counts, Fo, e_part, kin_part,
                       th);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

using LaunchFn = hpf_status_t (*)(const float3*, float3*, float3*, const uint8_t*, int64_t, const TileK&, int,
                                  const float3*, const int32_t*, int, float, float, const BoxK&, const float*, float,
                                  const uint32_t*, unsigned long long*, unsigned long long*, float3*, double*,
                                  double*, const ThermoK&, hipStream_t);

template <bool kPipe, bool kNT>
static LaunchFn scatter_launch_fn(bool wide, bool thermo, bool r0z)
{
    if (wide)
        return launch_advance_scatter_t<true, kASThreadsWide, kPipe, false, kNT>;
    if (r0z)
        return thermo ? launch_advance_scatter_t<true, kASThreadsDefault, kPipe, true, kNT>
                      : launch_advance_scatter_t<true, kASThreadsDefault, kPipe, false, kNT>;
    return thermo ? launch_advance_scatter_t<false, kASThreadsDefault, kPipe, true, kNT>
                  : launch_advance_scatter_t<false, kASThreadsDefault, kPipe, false, kNT>;
}

hpf_status_t launch_advance_scatter(const float* R, float* R_next, float* Vel, const uint8_t* T, int64_t N,
                                    const TileK& tk, int K, const float* G, const int32_t* bonds, int D, float k,
                                    float r0, const BoxK& box, const float* inv_mass, float dt,
                                    const uint32_t* cell_start, unsigned long long* partials,
                                    unsigned long long* counts, float* F_out, double* e_part, double* kin_part,
                                    const ThermoK& th, hipStream_t s)
{
    auto* Rp = reinterpret_cast<const float3*>(R);
    auto* Rn = reinterpret_cast<float3*>(R_next);
    auto* Vp = reinterpret_cast<float3*>(Vel);
    auto* Gp = reinterpret_cast<const float3*>(G);
    auto* Fo = reinterpret_cast<float3*>(F_out);
    // the software-pipelined bead loop serves bond tables of up to kPreBonds rows and
    // gradient meshes of up to kBufMeshBytes
    const bool pipe = D <= kPreBonds && (int64_t)K * tk.m.nm * 12 <= kBufMeshBytes;
    const bool thermo = th.thr != 0, r0z = r0 == 0.0f;
    // A deposit box of more than 80 KiB (16-cell bricks) leaves room for one workgroup per
    // CU: with r0 = 0 and no thermostat the pass then takes 768 threads (3 waves per SIMD;
    // 1024 threads would cap it at 128 VGPRs, which spills); the others keep 512.
    const bool wide = r0z && !thermo && sizeof(unsigned long long) * (size_t)K * tk.P * tk.P * tk.P > 80 * 1024;
    const int64_t box_bytes = (int64_t)sizeof(unsigned long long) * K * tk.P * tk.P * tk.P * tk.ntiles;
    const bool nt = pipe && streamed_bytes(N, D, K, tk.m, box_bytes) > kStreamHintBytes;
    const LaunchFn launch = pipe ? (nt ? scatter_launch_fn<true, true>(wide, thermo, r0z)
                                       : scatter_launch_fn<true, false>(wide, thermo, r0z))
                                 : scatter_launch_fn<false, false>(wide, thermo, r0z);
    return launch(Rp, Rn, Vp, T, N, tk, K, Gp, bonds, D, k, r0, box, inv_mass, dt, cell_start, partials, counts, Fo,
                  e_part, kin_part, th, s);
}

// Andersen collisions of time level *th.step on every bead (after the second half
// kick), and optionally the kinetic-energy and momentum partials of the result.
__global__ __launch_bounds__(kPThreads) void k_andersen(float3* __restrict__ Vel, const float* __restrict__ inv_mass,
                                                        int64_t N, ThermoK th, double* __restrict__ kin_part)
{
    __shared__ double scratch[kPThreads / kWave];
    const BeadWalk w = bead_walk(N);
    clear_unused_slots(kin_part, 4);
    const uint64_t tstep = thermo_step(th);
    KinAcc acc;
    FOR_BEADS(w, i) {
        const float im = inv_mass ? inv_mass[i] : 1.0f;
        float3 v = Vel[i];
        if (th.thr && andersen_collide(th, tstep, th.tag[i], im, v))
            Vel[i] = v;
        acc.add(v, im);
    }
    if (kin_part)
        acc.store(kin_part, w.block, scratch);
}

hpf_status_t launch_andersen(float* Vel, const float* inv_mass, int64_t N, const ThermoK& th, double* kin_part,
                             hipStream_t s)
{
    if (N == 0 && !kin_part)
        return HPF_OK;
    const int64_t nb = bead_blocks(N, kin_part ? HPF_NPART : (1 << 20));
    hipLaunchKernelGGL(k_andersen, dim3((unsigned)nb), dim3(kPThreads), 0, s, reinterpret_cast<float3*>(Vel),
                       inv_mass, N, th, kin_part);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

hpf_status_t launch_scatter_finish(const unsigned long long* partials, const TileK& tk, int K,
                                   unsigned long long* counts, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter_sum<true>, dim3((unsigned)tk.ntiles), sum_block(tk.ntiles), 0, s, partials, tk, K,
                       counts);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

// ------------------------------------------------------------- reduction ---

// out[c] = sum of part[c][0..HPF_NPART) in a fixed order (one block per c):
// each thread adds its slots j, j + 1024, ... (all loads issued first), then the
// block sum.
constexpr int kRedThreads = 1024;
static_assert(HPF_NPART % kRedThreads == 0, "partial slots must fill the reduction block");

__global__ __launch_bounds__(kRedThreads) void k_reduce_partials(const double* __restrict__ part,
                                                                 double* __restrict__ out)
{
    __shared__ double scratch[kRedThreads / kWave];
    const double* p = part + (int64_t)blockIdx.x * HPF_NPART;
    constexpr int kPer = HPF_NPART / kRedThreads;
    double v[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        v[j] = p[threadIdx.x + j * kRedThreads];
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        t += v[j];
    const double s = block_sum(t, scratch);
    if (threadIdx.x == 0)
        out[blockIdx.x] = s;
}

hpf_status_t launch_reduce_partials(const double* part, int ncomp, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_partials, dim3(ncomp), dim3(kRedThreads), 0, s, part, out);
    return hipGetLastError() == hipSuccess ? HPF_OK : HPF_EHIP;
}

}  // namespace hpf
