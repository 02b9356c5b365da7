/*
 * tslb.h - C ABI of the MI355X (gfx950) moment-only, high-order thread-safe
 * lattice Boltzmann library.
 *
 * Method: Montessori et al., "High-order thread-safe lattice Boltzmann model
 * for HPC turbulent flow simulations", arXiv:2401.17074.  Each time step,
 * every fluid node x pulls the moments (rho, u, Pi^neq) of its 27 D3Q27
 * upstream neighbours x - c_i, rebuilds each population as the third-order
 * Hermite equilibrium (Section 2.2, Eq. (eqts)) plus (1 - omega) times the
 * non-equilibrium part rebuilt by the Hermite recursion (Eq. (noneqts)), adds
 * the local body-force term (Section 3.1), and sums the new moments (the full
 * update of Section 2.2).  Only the ten moments are stored (Section 2.2, the
 * storage remark), double-buffered, structure-of-arrays.
 *
 * Conventions shared by every call
 *  - Grid: nx * ny * nz nodes, node index n = x + nx * (y + ny * z).
 *  - Field arrays are structure-of-arrays, x fastest: u is 3N floats
 *    (u_x block, u_y block, u_z block); Pi^neq is 6N floats ordered
 *    xx, yy, zz, xy, xz, yz; a force field is 3N floats like u.
 *  - Node classes follow from coordinates and the face kinds: a node on a
 *    TSLB_WALL face layer is solid (half-way bounce-back, walls win); a node
 *    on a TSLB_INLET / TSLB_OUTLET face layer is a ghost whose moments are
 *    refilled from the nearest interior node after every step (Section 2.3,
 *    Eq. (neq_final)); every other node is fluid and is updated.
 *  - Pointers are borrowed for the duration of the call; the handle owns its
 *    state buffers.  `stream` is a hipStream_t passed as void* (NULL = the
 *    default stream).  Calls are asynchronous on that stream unless they say
 *    otherwise.
 *  - Every call returns TSLB_OK (0) or a negative TSLB_E_* code; the message
 *    of the last failure on the calling thread is tslb_last_error().  No C++
 *    exception crosses this interface.
 */
#ifndef TSLB_H
#define TSLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tslb_ctx *tslb_handle; /* opaque, owned by the library */

enum { TSLB_D3Q27 = 27, TSLB_D3Q19 = 19, TSLB_D2Q9 = 9 };   /* lattices (Section 2.1 and 2.2) */
enum { TSLB_FP32 = 0, TSLB_FP16 = 1, TSLB_BF16 = 2 };       /* moment storage; compute is FP32 */
enum { TSLB_PERIODIC = 0, TSLB_WALL = 1, TSLB_INLET = 2, TSLB_OUTLET = 3 }; /* face kinds */
enum { TSLB_DEVICE = 1, TSLB_RHO_DEVIATION = 2 };           /* set/get flags */
enum { TSLB_OBJ_KINETIC_ENERGY = 0, TSLB_OBJ_WALL_SHEAR = 1 }; /* adjoint objectives */
enum { TSLB_STATS_PROFILE = 1, TSLB_STATS_FIELD = 2 };      /* statistics kinds (bit set) */
#define TSLB_MAX_NODES (1LL << 30)                           /* nx*ny*nz must stay below this */
enum {
    TSLB_OK = 0,
    TSLB_E_INVALID = -1,     /* bad argument (tau <= 1/2, dims, unpaired periodic faces, ...) */
    TSLB_E_UNSUPPORTED = -2, /* valid request this library does not provide */
    TSLB_E_NOMEM = -3,       /* device allocation failed */
    TSLB_E_HIP = -4,         /* a HIP runtime call failed */
    TSLB_E_UNSTABLE = -5     /* tslb_reduce met a NaN or Inf */
};

/* Boundary and storage description.
 *  face[6]         kinds of the faces -x, +x, -y, +y, -z, +z.  PERIODIC faces
 *                  come in pairs; a non-periodic axis needs at least 3 nodes.
 *  inlet_*         for TSLB_INLET faces: nodes of the face layer inside the
 *                  disc |(t1, t2) - inlet_center| <= inlet_radius (t1 < t2 are
 *                  the two transverse axes in x, y, z order) get
 *                  u = inlet_u + inlet_noise * |inlet_u| * xi per component,
 *                  xi drawn afresh at every level t from the SplitMix64 stream
 *                  of `seed` (see inlet_noise_kind); rho and Pi^neq come from the interior
 *                  neighbour.  The rest of an inlet face behaves as an outlet
 *                  (all ten moments copied from the interior neighbour).
 *  storage         TSLB_FP32 / TSLB_FP16 / TSLB_BF16 for the stored moments.
 *  scale[3]        power-of-two factors applied before rounding to 16 bits:
 *                  stored = (rho - 1) * scale[0], u * scale[1], Pi * scale[2].
 *                  0 selects the default for the storage kind (1 for FP32 and
 *                  BF16; 2^12, 2^12, 2^16 for FP16, which keeps |rho - 1| and
 *                  |u| below 16 and |Pi| below 1 clear of overflow and small
 *                  values clear of subnormals).  Ignored for FP32.
 *  order           Hermite order of the rebuilt populations: 3 (or 0, the
 *                  default) is the third-order equilibrium plus the recursive
 *                  non-equilibrium part of Section 2.2; 2 is the regularised
 *                  second-order collision of Eq. (fullstrcoll) (equilibrium of
 *                  Eq. (lbequil), non-equilibrium part projected on H2 only).
 *                  The adjoint and rollout calls need order 3.
 *  inlet_noise_kind 0: xi uniform in [-1, 1), the top 24 bits of output
 *                  k = 1 + 3 (t N + n) + component (node n, level t) mapped
 *                  to 2 (h >> 40) 2^-24 - 1.  1: xi standard Gaussian (the
 *                  time-varying Gaussian inflow noise of Section 3.2), the
 *                  Box-Muller transform sqrt(-2 ln v1) cos(2 pi v2) of
 *                  v1 = ((h1 >> 40) + 1) 2^-24 and v2 = (h2 >> 40) 2^-24 from
 *                  outputs k1 = 1 + 6 (t N + n) + 2 component and k1 + 1.   */
typedef struct {
    int face[6];
    float inlet_u[3];
    float inlet_center[2];
    float inlet_radius;
    float inlet_noise;
    uint64_t seed;
    int storage;
    float scale[3];
    int order;
    int inlet_noise_kind;
} tslb_bc;

/* Create a solver on an nx*ny*nz grid (Section 2.2 update).
 * lattice: TSLB_D3Q27; TSLB_D3Q19 (the 19 rest, face and edge velocities,
 *   weights 1/3, 1/18, 1/36: the reconstruction keeps the third-order
 *   Hermite content this lattice supports, i.e. the three pairs
 *   (xxy, yzz), (xzz, xyy), (yyz, xxz) projected on their sums and
 *   differences with the lattice's own norms 2 cs^6 and 6 cs^6, and no xyz
 *   term; tiled kernel only, no adjoint); or TSLB_D2Q9 (the two-dimensional counterpart: the
 *   same reconstruction on the nine-velocity tensor-product lattice; needs
 *   nz = 1, periodic z faces and zero z components of force and inlet
 *   velocity; the state keeps the ten-field layout with u_z and the Pi
 *   components xz, yz, zz held at zero; one update kernel, no adjoint).
 * nx*ny*nz must stay below TSLB_MAX_NODES = 2^30 (the kernels address each
 *   field with 32-bit byte offsets; 2^30 nodes hold 86 GB of FP32 state).
 * tau: relaxation time, nu = (tau - 1/2) / 3 (Section 2), must exceed 1/2.
 * force: uniform body acceleration g (Section 3.1 forcing), may be NULL (0).
 * bc: may be NULL (all faces periodic, FP32 storage).
 * Allocates two state buffers on the current HIP device, sets the rest
 * state rho = 1, u = 0, Pi^neq = 0 at level t = 0, and synchronises.
 * Errors: TSLB_E_INVALID (also for too many nodes), TSLB_E_UNSUPPORTED
 * (other lattices), TSLB_E_NOMEM.                                            */
int tslb_create(int nx, int ny, int nz, int lattice, float tau, const float force[3], const tslb_bc *bc,
                tslb_handle *out);

/* Free the buffers of h (synchronises the device first).  NULL is a no-op. */
int tslb_destroy(tslb_handle h);

/* Overwrite the state at the current level with rho (N), u (3N) and Pi^neq
 * (6N, or NULL for zero): the ten hydrodynamic moments that are the only
 * stored variables of the scheme (Section 2.2, the storage remark; Pi^neq is
 * the pre-collision non-equilibrium second moment the reconstruction of
 * Eq. (noneqts) starts from).  flags: TSLB_DEVICE if the arrays are device
 * memory (else host; the call then synchronises the stream),
 * TSLB_RHO_DEVIATION if `rho` holds rho - 1.  Values are rounded to the
 * storage format; ghost layers are then refilled from the interior (so input
 * ghost values are ignored) and solid (wall) nodes are stored as the rest
 * state rho = 1, u = 0, Pi = 0 whatever the input holds.                   */
int tslb_set_moments(tslb_handle h, const float *rho, const float *u, const float *pineq, int flags,
                     void *stream);

/* Read the current state, the moments of Section 2.2 (rho, u, Pi^neq) at
 * level t (all nodes; ghosts hold their fill values of Section 2.3, solid
 * nodes the rest state).  Any output pointer may be NULL.  Same flags as
 * tslb_set_moments; host reads synchronise the stream.                      */
int tslb_get_moments(tslb_handle h, float *rho, float *u, float *pineq, int flags, void *stream);

/* Use a per-node body-acceleration field g (3N floats, device memory,
 * copied into the handle) instead of the uniform force; NULL returns to the
 * uniform force given at creation.  The forcing is the local term of
 * Section 3.1, w_i rho c_i.g / cs2 added to every population a node emits,
 * with rho and g of the emitting node (no half-force velocity shift), so a
 * step changes the total momentum by exactly sum rho g over fluid nodes.
 * The field also parameterises the adjoint (tslb_adjoint_step dg_accum).
 * Errors: TSLB_E_NOMEM (first use allocates 3N floats).                    */
int tslb_set_force_field(tslb_handle h, const float *g, void *stream);

/* Relaxation time per z plane: tau_z holds nz values (host memory, each
 * > 1/2), copied into the handle; every node then relaxes with the value of
 * its own plane, in the update and in the adjoint.  This carries the outlet
 * sponge of the jet benchmark (Section 3.2), where the viscosity grows
 * towards the outflow face.  NULL returns to the uniform tau of creation.
 * Synchronises the stream.  Errors: TSLB_E_INVALID for a value <= 1/2 or not
 * finite (the profile is then unchanged), TSLB_E_NOMEM.                     */
int tslb_set_relaxation_profile(tslb_handle h, const float *tau_z, void *stream);

/* Advance nsteps time steps (Section 2.2 update, then the ghost refill of
 * Section 2.3 for the new level).  Asynchronous.  nsteps >= 0.               */
int tslb_step(tslb_handle h, int nsteps, void *stream);

/* tslb_step with per-launch timing, for profiling: HIP events recorded on
 * `stream` around every launch give ms[0] = summed device time of the main
 * update kernel launches and ms[1] = summed time of the per-step auxiliary
 * launches (wall fix-up, ghost refill).  Synchronises the stream.  The
 * events add a few microseconds between launches, so tslb_step is the one to
 * time whole runs with.  1 <= nsteps <= 100000.                             */
int tslb_step_timed(tslb_handle h, int nsteps, double ms[2], void *stream);

/* Current level t (steps taken since creation, or the last tslb_set_time). */
int64_t tslb_get_time(tslb_handle h);
int tslb_set_time(tslb_handle h, int64_t t);

/* FP64 sums over fluid nodes of the current state: out[0] = sum rho,
 * out[1..3] = sum rho u, out[4] = 1/2 sum rho |u|^2 (conservation checks of
 * Section 2).  Synchronises the stream.  Returns TSLB_E_UNSTABLE (with out
 * still written) if any stored fluid moment is NaN or Inf.                   */
int tslb_reduce(tslb_handle h, double out[5], void *stream);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the sums of tslb_reduce, in the same fixed order and bit-identical to it,
 * with no allocation, no host copy and no synchronisation.
 *  out_dev  device pointer to TSLB_REDUCE_VALUES doubles, written
 *           asynchronously on `stream`: mass, momentum (3), kinetic energy,
 *           the count of fluid nodes holding NaN/Inf moments (as a double;
 *           this call does not return TSLB_E_UNSTABLE) and the wall-shear
 *           objective of tslb_objective.
 * The per-block partial sums go to one fixed library array per GPU
 * (TSLB_NOALLOC_REDUCE_BLOCKS x 7 doubles = 56 KiB, held until the process
 * ends; every partial is rewritten by each call).  Calls that overlap on one
 * GPU (other streams or threads) race on that array: serialise them.
 * Errors: TSLB_E_INVALID (NULL handle or out_dev; a reduction wider than the
 * fixed array), TSLB_E_HIP.                                                  */
#define TSLB_REDUCE_VALUES 7
#define TSLB_NOALLOC_REDUCE_BLOCKS 1024
int tslb_reduce_noalloc(tslb_handle h, double *out_dev, void *stream);

/* Raw state snapshots (for checkpoints and the adjoint): the state is
 * tslb_state_bytes(h) bytes of device memory holding the ten stored fields
 * in storage format, SoA, field 0 = (rho - 1) * scale[0].  dst/src are
 * device pointers; asynchronous D2D copies.  Loading does not refill ghosts. */
size_t tslb_state_bytes(tslb_handle h);
int tslb_save_state(tslb_handle h, void *dst, void *stream);
int tslb_load_state(tslb_handle h, const void *src, void *stream);

/* Hand the two state buffers to caller-owned device memory (e.g. tensors
 * from PyTorch's allocator): buf0 and buf1 each hold tslb_state_bytes(h)
 * bytes, 256-byte aligned, distinct, on the handle's device, and must stay
 * alive until tslb_destroy or the next tslb_bind_state.  Both current
 * buffers are copied over (the current level into buf0, so wall and ghost
 * layers keep their contents), the stream is synchronised, and buffers the
 * library allocated itself are freed; bound buffers are never freed by the
 * library.  Errors: TSLB_E_INVALID (NULL, aliasing or misaligned buffers). */
int tslb_bind_state(tslb_handle h, void *buf0, void *buf1, void *stream);

/* Discrete adjoint (reverse-mode derivative) of one update step, the
 * transpose of the Section 2.2 update linearised at state_t:
 *   lam_t    = (dM_{t+1}/dM_t)^T lam_t1
 *   dg_accum += (dM_{t+1}/dg)^T lam_t1   (per-node force field; may be NULL)
 * state_t, state_t1: raw snapshots (tslb_save_state format) of levels t and
 * t+1 = step(state_t).  lam_t1, lam_t: 10N floats, SoA, one sensitivity per
 * stored moment (rho, u_x, u_y, u_z, Pi xx, yy, zz, xy, xz, yz); lam_t may
 * not alias lam_t1.  Uses tau, force and faces of h.
 * With inflow/outflow ghost layers (Section 2.3, Eq. (neq_final)) a step is
 * the update of the fluid nodes followed by the refill of the new level's
 * ghosts from the interior nodes they copy; the ghost values of level t are
 * inputs like any other node (lam_t is nonzero there: ghosts emit).  The
 * refill is transposed first, IN PLACE on lam_t1: each ghost node's
 * sensitivities are added to the node it copies (rho and Pi^neq only on an
 * inlet disc, whose velocity is imposed) and then cleared.  Without ghost
 * layers lam_t1 is only read.
 * Errors: TSLB_E_UNSUPPORTED unless storage is FP32, the order is 3 and the
 * lattice D3Q27.                                                            */
int tslb_adjoint_step(tslb_handle h, const void *state_t, const void *state_t1, float *lam_t1, float *lam_t,
                      float *dg_accum, void *stream);

/* Seed of the adjoint: lam = dL/dM for the objective at a raw state
 * (TSLB_OBJ_KINETIC_ENERGY: L = 1/2 sum_fluid rho |u|^2, so lam_rho =
 * |u|^2 / 2, lam_u = rho u, lam_Pi = 0; zero on non-fluid nodes.
 * TSLB_OBJ_WALL_SHEAR: the x-directed viscous force on the walls normal to
 * y and z, L = sum over fluid nodes next to such a wall face f of
 * s_f sigma_xd, d the face's normal axis, s_f = +1 on the low and -1 on the
 * high face, sigma = -(1 - omega/2) Pi^neq the viscous stress of the BGK
 * update (Section 2); lam is -s_f (1 - omega/2) on Pi_xd of those nodes and
 * zero elsewhere).                                                          */
int tslb_adjoint_seed(tslb_handle h, const void *state, int objective, float *lam, void *stream);

/* Value of an objective (as for tslb_adjoint_seed) at the current level,
 * summed in FP64 in a fixed order.  Synchronises the stream.  Returns
 * TSLB_E_UNSTABLE (with *out still written) if any fluid moment is NaN/Inf. */
int tslb_objective(tslb_handle h, int objective, double *out, void *stream);

/* Checkpointed rollout for gradients (recompute-every-K scheme).
 * tslb_rollout_workspace_bytes: device bytes needed for nsteps with a
 * checkpoint every `every` steps.  tslb_rollout_forward advances the
 * handle by nsteps, storing a raw snapshot in `ws` at the start of every
 * segment.  tslb_rollout_backward then takes lam (10N, in: dL/dM at the
 * final level, out: dL/dM at the initial level) and accumulates dL/dg into
 * dg_accum (3N, may be NULL), recomputing each segment once from its
 * checkpoint (each level computed straight into the workspace) and running
 * tslb_adjoint_step backwards through it; the handle's state and level are
 * left as they were.  With ghost layers the recomputed levels are refilled
 * like the forward ones, and lam on return is the gradient with respect to
 * the initial level's interior (its ghosts were refilled from it: their
 * sensitivities are folded in and cleared).                                  */
size_t tslb_rollout_workspace_bytes(tslb_handle h, int nsteps, int every);
int tslb_rollout_forward(tslb_handle h, int nsteps, int every, void *ws, size_t ws_bytes, void *stream);
int tslb_rollout_backward(tslb_handle h, int nsteps, int every, void *ws, size_t ws_bytes, float *lam,
                          float *dg_accum, void *stream);

/* Velocity statistics of the turbulence benchmarks, accumulated on the
 * device in FP64 (Section 3.1: averages over the homogeneous directions and
 * time; Section 3.2: time averages of the jet).
 *  kinds  TSLB_STATS_PROFILE: for every index j along `axis` (0 x, 1 y,
 *         2 z), sums over the fluid nodes of plane j of 1, u_x, u_y, u_z,
 *         the products u_a u_b in the order xx, yy, zz, xy, xz, yz, and
 *         u_x^3, u_y^3, u_z^3 (13 values per plane, 13 n_axis doubles).
 *         TSLB_STATS_FIELD: per-node sums of u_a and u_a u_b (9 N doubles).
 * tslb_stats_begin zeroes the sums and the sample count (allocating on first
 * use; TSLB_E_NOMEM) and keeps `axis` for PROFILE; tslb_stats_sample adds
 * the current level as one sample (asynchronous).  The central moments
 * <u'_a u'_b> = <u_a u_b> - U_a U_b and <u'^3> = <u^3> - 3 U <u^2> + 2 U^3
 * follow from the sums; S_2 = <u'u'>/u_tau^2 and S_3 = <u'^3>/<u'^2>^(3/2)
 * as in Section 3.1.  Errors: TSLB_E_INVALID (kinds 0 or unknown, axis out
 * of range, no sample yet for the read calls).                               */
int tslb_stats_begin(tslb_handle h, int kinds, int axis, void *stream);
int tslb_stats_sample(tslb_handle h, void *stream);

/* Profile sums (host array of 13 n_axis doubles, row j = plane j) and the
 * number of samples (may be NULL).  Synchronises the stream.                */
int tslb_stats_profile(tslb_handle h, double *sums, int64_t *nsamples, void *stream);

/* From the FIELD sums: per-node means <u_a> (3N floats, SoA) and
 * covariances <u'_a u'_b> (6N floats, xx, yy, zz, xy, xz, yz), written to
 * device memory; either pointer may be NULL.  Asynchronous.                 */
int tslb_stats_field(tslb_handle h, float *mean_u, float *cov, void *stream);

/* Jet diagnostics from the FIELD means (Section 3.2): for every
 * cross-section j along `axis`, the nodes are grouped by k = floor(r), r
 * their distance to the axis point `center` (its two transverse
 * coordinates in x, y, z order, inside the cross-section); bin k has mean
 * radius rbar_k and mean axial velocity P_k.  uc[j] = P_0 (the centreline
 * velocity: nodes within one spacing of the axis) and rhalf[j] = the
 * half-width, interpolated linearly between the first bin k >= 1 with
 * P_k <= uc[j] / 2 and the nearest non-empty bin before it (-1 if none).
 * uc and rhalf are device arrays of n_axis floats.  Asynchronous.
 * Errors: TSLB_E_INVALID (no FIELD samples, centre outside the
 * cross-section, cross-section too wide for the LDS bins).                  */
int tslb_stats_jet(tslb_handle h, int axis, const float center[2], float *uc, float *rhalf, void *stream);

/* Kernel selection for the update and the adjoint step:
 *  0  the LDS-tiled z-marching kernels (default);
 *  1  the direct one-thread-per-node kernels (cross-checks);
 *  2  the population layout of the paper's own GPU code (the memory-footprint
 *     remark of Section 2.2): a push pass writes every node's 27 populations
 *     into one population set, a second pass sums them into the moments.
 *     Allocates 27 N floats on first selection (kept until tslb_destroy;
 *     TSLB_E_NOMEM if that fails, the variant then stays unchanged); the
 *     adjoint step uses the tiled kernel.
 * All compute the same update up to FP32 summation order.                   */
int tslb_set_kernel(tslb_handle h, int variant);

/* Message of the last failed call on this thread ("" if none). */
/* Bandwidth reference (not part of the method): copies `bytes` from src to
 * dst, both device pointers on the current device, with a plain streaming
 * kernel (each 16-byte word read once and written once), asynchronously on
 * `stream`.  Its rate is the practical read+write ceiling that the update's
 * rate is compared with, and its HBM counter readings calibrate the
 * counters.  Errors: TSLB_E_INVALID (NULL, overlapping buffers, a size or
 * address that is not a multiple of 16), TSLB_E_HIP.                        */
int tslb_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

const char *tslb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TSLB_H */
