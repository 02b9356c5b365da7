// Host-side context of a TSLB solver handle and the launchers each kernel
// translation unit exports to the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
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
    // Wall-adjacent fluid nodes: the tiled update leaves their raw moment
    // sums here (FP32, ten per node) and a fix-up pass adds the bounced-back
    // populations.  The layer next to wall face f starts at wall_off[f]
    // nodes (-1: face f is not a wall).
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

// Launchers (stream-ordered, no synchronisation).  `storage` selects the
// stored format (0 FP32, 1 FP16, 2 BF16); buffers are the raw state arrays.
hipError_t launch_update_direct(int storage, const void* in, void* out, const StepParams& p, hipStream_t s);
hipError_t launch_update_poplayout(int storage, const void* in, void* out, float* pop, const StepParams& p,
                                   hipStream_t s);
hipError_t launch_update_tiled(int storage, const void* in, void* out, const StepParams& p, hipStream_t s);
hipError_t launch_update_d2q9(int storage, const void* in, void* out, const StepParams& p, hipStream_t s);
int stats_blocks_per_plane(const Geometry& g, int axis);
int stats_jet_bins(const Geometry& g, int axis, float c1, float c2);
hipError_t launch_stats_profile(int storage, const void* st, double* part, double* sums, const StepParams& p,
                                int axis, hipStream_t s);
hipError_t launch_stats_field(int storage, const void* st, double* fs, const StepParams& p, hipStream_t s);
hipError_t launch_stats_field_moments(const double* fs, long long N, double inv_ns, float* mean, float* cov,
                                      hipStream_t s);
hipError_t launch_stats_jet(const double* fs, const Geometry& g, int axis, float c1, float c2, double inv_ns,
                            float* uc, float* rhalf, hipStream_t s);
// Completes the wall-adjacent nodes after launch_update_tiled (walls only).
hipError_t launch_wall_fixup(int storage, const void* in, void* out, const StepParams& p, hipStream_t s);
hipError_t launch_ghost_fill(int storage, void* st, const StepParams& p, const InletParams& q, int64_t t,
                             hipStream_t s);
hipError_t launch_pack(int storage, const float* rho, const float* u, const float* pi, int rho_dev, void* st,
                       const StepParams& p, hipStream_t s);
hipError_t launch_unpack(int storage, const void* st, float* rho, float* u, float* pi, int rho_dev,
                         const StepParams& p, hipStream_t s);
// FP64 partial sums: writes 5 sums + 1 non-finite count (as double) into out6 (device).
hipError_t launch_reduce(int storage, const void* st, double* partials, int nblocks, double* out6,
                         const StepParams& p, hipStream_t s);
hipError_t launch_adjoint_seed(const float* st, float* lam, const StepParams& p, hipStream_t s);
hipError_t launch_adjoint_step(const float* st0, const float* st1, const float* lam1, float* lam0, float* dg,
                               const StepParams& p, hipStream_t s);
hipError_t launch_adjoint_tiled(const float* st0, const float* st1, const float* lam1, float* lam0, float* dg,
                                const StepParams& p, hipStream_t s);

}  // namespace tslb

struct tslb_ctx {
    int device;
    tslb::StepParams p;
    tslb::InletParams inlet;
    int storage;
    size_t elem_bytes;       // bytes per stored value
    void* buf[2];            // ping-pong raw states, 10 N values each
    int cur;                 // index of the buffer holding the current level
    float* gfield;           // owned copy of the per-node force field (or null)
    float* staging;          // device staging for host set/get (10 N floats, lazily)
    double* red_partials;    // reduction partials
    double* red_out;         // 6 doubles
    int red_blocks;
    int64_t t;               // current level
    int kernel;              // 0 tiled, 1 direct, 2 population layout
    int lattice;             // 27 or 9
    float* pop;              // 27 N populations of the population-layout variant (lazily)
    float* omo_z;            // owned per-plane 1 - omega (or null)
    // velocity statistics (FP64 sums, lazily allocated)
    int stats_kinds;         // TSLB_STATS_* bits enabled by the last begin
    int stats_axis;          // profile axis
    int64_t stats_samples;
    double* stats_prof;      // 13 n_axis sums
    double* stats_part;      // per-block partials of one profile sample
    int stats_prof_axis;     // axis the two buffers above are sized for (-1: none)
    double* stats_field;     // 9 N sums
    bool has_ghosts;
};
