// Andersen thermostat on the device (Integration methods section: NVT by the
// Andersen thermostat). At time level n a bead collides with the heat bath with
// probability p and takes a fresh Maxwell velocity at kT. Every random number
// comes from the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and
// Shaw, SC'11) keyed on (tag, n), so a bead's draws do not depend on where it is
// stored, on the launch shape or on which pass applies them.
#pragma once

#include "hpf_common.hpp"

namespace hpf {

// Thermostat as passed to kernels (by value). thr = 0 switches it off.
struct ThermoK {
    uint32_t thr;            // collision when the 24-bit uniform integer is below floor(p 2^24)
    float kT;
    uint32_t key0, key1;     // generator key (the seed)
    const int64_t* step;     // device: time level of the collisions
    const int32_t* tag;      // device: bead tags (the generator's per-bead counter word)
    uint32_t tag_off;        // added to every tag in that counter word
};

// Ten Philox rounds: counter words 0 and 2 are multiplied by the round constants into
// 64-bit products (high and low halves); the high halves are mixed with words 1 and 3 and
// the key, which advances by the two Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// The bead with tag `tag` (counter word tag + tag_off) at time level `step`: false if
// it does not collide; else true with v.xyz replaced by sqrt(kT im) (g0, g1, g2), the three standard normal deviates of
// two Box-Muller pairs on 24-bit uniforms (u = (r >> 8) 2^-24, shifted to (0, 1] where a
// logarithm is taken): g0, g1 from words 1, 2 of counter (tag, step, 0) and g2 from its
// word 3 and word 0 of counter (tag, step, 1).
__device__ __forceinline__ bool andersen_collide(const ThermoK& th, uint64_t step, int32_t tag, float im,
                                                 float3& v)
{
    uint4 c = make_uint4((uint32_t)tag + th.tag_off, (uint32_t)step, (uint32_t)(step >> 32), 0u);
    const uint4 r = philox4x32_10(c, th.key0, th.key1);
    if ((r.x >> 8) >= th.thr)
        return false;
    c.w = 1u;
    const uint32_t r4 = philox4x32_10(c, th.key0, th.key1).x;
    const float two_pi = 6.28318530717958647692f;
    const float u1 = (float)((r.y >> 8) + 1u) * 0x1p-24f;
    const float u2 = (float)(r.z >> 8) * 0x1p-24f;
    const float u3 = (float)((r.w >> 8) + 1u) * 0x1p-24f;
    const float u4 = (float)(r4 >> 8) * 0x1p-24f;
    const float rad1 = sqrtf(-2.0f * logf(u1));
    const float rad2 = sqrtf(-2.0f * logf(u3));
    float s1, c1;
    sincosf(two_pi * u2, &s1, &c1);
    const float sd = sqrtf(th.kT * im);
    v.x = sd * (rad1 * c1);
    v.y = sd * (rad1 * s1);
    v.z = sd * (rad2 * cosf(two_pi * u4));
    return true;
}

// Time level of this launch's collisions (every thread reads the same word).
__device__ __forceinline__ uint64_t thermo_step(const ThermoK& th)
{
    return th.thr ? (uint64_t)*th.step : 0ull;
}

}  // namespace hpf
