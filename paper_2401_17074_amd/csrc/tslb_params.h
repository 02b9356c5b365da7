// Parameters the kernels receive by value: the per-step parameters of the
// update and the inflow description of the ghost refill.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tslb_device.h"

namespace tslb {

// Runtime parameters every update launch needs.
struct StepParams {
    Geometry geo;
    float one_minus_omega;   // 1 - 1/tau
    int order;               // Hermite order of the rebuilt populations (2 or 3)
    int dims;                // 3 (D3Q27, D3Q19) or 2 (D2Q9: u_z and the z components of Pi stay zero)
    int lattice;             // 27, 19 or 9
    const float* omo_z;      // optional 1 - omega per z plane (nz floats), else one_minus_omega
    float force[3];          // uniform acceleration (used when gfield == nullptr)
    const float* gfield;     // optional per-node acceleration, 3N SoA
    float scale[3];          // storage scales (drho, u, Pi); 1 for FP32
    float inv_scale[3];
    // Wall-adjacent fluid nodes when the tiled update is built without the
    // in-kernel bounce-back (TSLB_FUSED_WALLS=0): it leaves their raw moment
    // sums here (FP32, ten per node) and a fix-up launch adds the
    // bounced-back populations.  The layer next to wall face f starts at
    // wall_off[f] nodes (-1: face f is not a wall).
    float* wall_side;
    long long wall_off[6];
    long long wall_nodes;
    // Work list of the tiled update (see tile::Schedule): sched_grid blocks,
    // sched_nseg entries {tile column, z begin, z end, 0} per block.
    const int4* sched;
    int sched_grid, sched_nseg;
};

// Inflow description for the ghost refill (Section 2.3).
struct InletParams {
    int face_kind[6];
    float u[3];
    float center[2];
    float radius2;
    float amp;               // noise * |u|
    uint64_t seed;
    int noise_kind;          // 0 uniform in [-1, 1), 1 standard Gaussian
};

// SplitMix64 output k of the stream seeded with `seed` (Steele, Lea and
// Flood, 2014): mix(seed + k * golden gamma).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int face_layer(const Geometry& g, int f) { return (f & 1) ? g.n[f >> 1] - 1 : 0; }

// Imposed velocity component a of ghost node n (coordinates c) at level t if
// the node lies on the disc of an inlet face: the top-hat velocity plus the
// seeded perturbation amp xi, xi uniform in [-1, 1) or standard Gaussian
// (Box-Muller) from SplitMix64 outputs indexed by (t N + n, a).  Returns
// false (and leaves u alone) off every inlet disc.
__device__ __forceinline__ bool inlet_velocity(const Geometry& g, const InletParams& q, int dims, int64_t t,
                                               long long n, const int c[3], float u[3]) {
    for (int f = 0; f < 6; ++f) {
        if (q.face_kind[f] != kInlet) continue;
        const int e = f >> 1;
        if (c[e] != face_layer(g, f)) continue;
        const int e1 = e == 0 ? 1 : 0, e2 = e == 2 ? 1 : 2;
        const float r1 = (float)c[e1] - q.center[0], r2 = (float)c[e2] - q.center[1];
        if (r1 * r1 + r2 * r2 > q.radius2) continue;
        const uint64_t tn = (uint64_t)t * (uint64_t)g.N + (uint64_t)n;
        for (int a = 0; a < dims; ++a) {
            float xi;
            if (q.noise_kind == 1) {
                // Box-Muller: sqrt(-2 ln v1) cos(2 pi v2), v1 in (0, 1], v2 in [0, 1)
                const uint64_t k = 1ull + 6ull * tn + 2ull * (uint64_t)a;
                const float v1 = (float)((splitmix64(q.seed, k) >> 40) + 1) * 0x1.0p-24f;
                const float v2 = (float)(splitmix64(q.seed, k + 1) >> 40) * 0x1.0p-24f;
                xi = sqrtf(-2.0f * logf(v1)) * cospif(2.0f * v2);
            } else {
                const uint64_t h = splitmix64(q.seed, 1ull + 3ull * tn + (uint64_t)a);
                xi = (float)(h >> 40) * 0x1.0p-24f * 2.0f - 1.0f;
            }
            u[a] = fmaf(q.amp, xi, q.u[a]);
        }
        return true;
    }
    return false;
}

// 1 - omega of the nodes of plane z.
__device__ __forceinline__ float omo_at(const StepParams& p, int z) {
    return p.omo_z ? p.omo_z[z] : p.one_minus_omega;
}

}  // namespace tslb
