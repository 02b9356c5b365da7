// Host-side context of a TSLB solver handle and the launchers each kernel
// translation unit exports to the C-ABI layer.
#pragma once
#include <vector>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tslb_device.h"
#include "tslb_params.h"

namespace tslb {

// Launchers (stream-ordered, no synchronisation).  `storage` selects the
// stored format (0 FP32, 1 FP16, 2 BF16); buffers are the raw state arrays.
hipError_t launch_update_direct(int storage, const void* in, void* out, const StepParams& p, hipStream_t s);
hipError_t launch_update_poplayout(int storage, const void* in, void* out, float* pop, const StepParams& p,
                                   hipStream_t s);
// Work list of the tiled update for grid g (host-side, see tile::Schedule).
hipError_t tiled_schedule(const Geometry& g, std::vector<int4>& seg, int& grid, int& nseg);
hipError_t launch_update_tiled(int storage, const void* in, void* out, const StepParams& p, hipStream_t s);
hipError_t launch_update_d2q9(int storage, const void* in, void* out, const StepParams& p, hipStream_t s);
bool tiled_uses_wall_side();  // the tiled update needs the wall side buffer and the fix-up launch
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
// x_done: the tiled update has written the ghost nodes of the x faces that
// lie on no other ghost face (inlet velocities are still imposed here)
hipError_t launch_ghost_fill(int storage, void* st, const StepParams& p, const InletParams& q, int64_t t,
                             int x_done, hipStream_t s);
// Does launch_update_tiled write those x-face ghost nodes for this grid and
// storage (rows of whole cache lines, no walls, no force field)?
bool tiled_writes_x_ghosts(int storage, const StepParams& p);
hipError_t launch_pack(int storage, const float* rho, const float* u, const float* pi, int rho_dev, void* st,
                       const StepParams& p, hipStream_t s);
hipError_t launch_unpack(int storage, const void* st, float* rho, float* u, float* pi, int rho_dev,
                         const StepParams& p, hipStream_t s);
// FP64 sums over fluid nodes, in a fixed order: mass, momentum (3), kinetic
// energy, the count of non-finite moments (as a double) and the wall shear
// objective, written to out6[kRedSums] (device).
constexpr int kRedSums = 7;
hipError_t launch_reduce(int storage, const void* st, double* partials, int nblocks, double* out6,
                         const StepParams& p, hipStream_t s);
hipError_t launch_stream_copy(const void* src, void* dst, long long n4, hipStream_t s);
// Transpose of the ghost refill, in place on lam (10 N floats): ghost nodes'
// sensitivities folded into the interior nodes they copy, then cleared.
hipError_t launch_ghost_fold(float* lam, const StepParams& p, const InletParams& q, hipStream_t s);
hipError_t launch_adjoint_seed(const float* st, float* lam, const StepParams& p, int objective, hipStream_t s);
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
    bool buf_owned;          // false once tslb_bind_state handed them to the caller
    int cur;                 // index of the buffer holding the current level
    float* gfield;           // owned copy of the per-node force field (or null)
    float* staging;          // device staging for host set/get (10 N floats, lazily)
    double* red_partials;    // reduction partials
    double* red_out;         // kRedSums doubles
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
    int4* sched;             // work list of the tiled update (owned)
};
