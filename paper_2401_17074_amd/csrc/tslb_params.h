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

// 1 - omega of the nodes of plane z.
__device__ __forceinline__ float omo_at(const StepParams& p, int z) {
    return p.omo_z ? p.omo_z[z] : p.one_minus_omega;
}

}  // namespace tslb
