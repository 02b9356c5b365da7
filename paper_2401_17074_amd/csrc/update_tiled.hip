// Tiled update kernel for gfx950: 2.5D z-march with the populations
// exchanged through LDS.
//
// The update of Section 2.2 pulls, for every node x and velocity c, the
// population that the upstream node x - c emits along c, rebuilt from that
// node's moments.  Here every node rebuilds its own 27 emitted populations
// exactly once per step and publishes them in LDS; each node then gathers
// the 27 arriving values from its neighbours.  The arithmetic per
// population is identical to the direct pull, only the sharing differs
// (thread-safe as in the paper: the level-t moments are read-only, the new
// level goes to a separate buffer).
//
// Per node the emitted populations are 216 w(c) P(c) with P a polynomial of
// degree <= 3 in the components of c.  Because c_a^3 = c_a on D3Q27, P has
// 17 monomial coefficients (1, c_a, c_a^2, c_a c_b, c_a^2 c_b, cx cy cz):
// they are formed once per node, the 27 values follow by a separable
// evaluation over z, then x, then y.  The arriving populations are reduced
// to moments by the transposed separable sums.
//
// Tile = TX x TY interior columns plus a one-node halo ring (extra waves)
// marching a segment of planes along z (plus one halo plane each side);
// one resident block per CU walks its list of segments, built on the host
// when the handle is created (tile::build_schedule).  A plane's emitted
// populations with (cx, cy) != (0, 0) go through LDS; the three with
// cx = cy = 0 stay in the thread.  Contributions to the output planes
// p - 1, p, p + 1 are accumulated in three rolling register sets.  The
// stored fields are loaded ahead of their use: one plane-step with 16-bit
// storage, two with FP32 storage.
#include "tslb_tiles.h"

namespace tslb {
namespace {

using namespace tile;


// MODE 0: plain output stores; 1: non-temporal ones; 2: non-temporal, and
// the fluid nodes next to x ghost faces also write those ghost nodes.
template <class S, bool WALLS, bool FIELD, int ORDER, int LAT, int MODE>
__global__ void __launch_bounds__(NTHREADS, TSLB_WAVES_PER_EU) update_tiled_kernel(const FieldPtrs<typename S::T> f, StepParams p,
                                                                   int tiles_x) {
    __shared__ float lds[NSLOT][LY][LX];
    // D3Q27: the populations travel without their weights, which the gather
    // applies for free (add_slice); D3Q19's weights are not separable
    constexpr bool kDeferWeights = LAT == 27;
    const Geometry& g = p.geo;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned plane_nodes = (unsigned)nx * (unsigned)ny;
    const bool pz = (g.periodic & 4) != 0;

    // this block's segments (uniform loads); an empty list ends the block
    // before any barrier
    const int4* __restrict__ segs = p.sched + (size_t)blockIdx.x * p.sched_nseg;
    int k = 0;
    int4 t = segs[0];
    if (t.x < 0) return;

    // thread -> LDS column (lx, ly); interior columns first, whole waves
    const int tid = threadIdx.x;
    int lx, ly;
    bool active = true;
    const bool interior = tid < NINT;
    if (interior) {
        lx = 1 + tid % TX;
        ly = 1 + tid / TX;
    } else {
        // halo columns, one kind per wave: the row below the tile (what it
        // sends into the tile has cy = +1), the row above (cy = -1), then the
        // four corners and the two side columns (cx = +1 on the left, -1 on
        // the right)
        static_assert(TX == 64 && 4 + 2 * TY <= 64 && NTHREADS == NINT + 192, "one wave per halo row");
        const int h = tid - NINT, lane = h & 63;
        if (h < 64) {
            lx = 1 + lane;
            ly = 0;
        } else if (h < 128) {
            lx = 1 + lane;
            ly = LY - 1;
        } else if (lane < 4) {
            lx = (lane & 1) ? LX - 1 : 0;
            ly = (lane & 2) ? LY - 1 : 0;
        } else if (lane < 4 + 2 * TY) {
            const int k = lane - 4;
            lx = (k < TY) ? 0 : LX - 1;
            ly = 1 + (k % TY);
        } else {
            lx = 0;
            ly = 0;
            active = false;
        }
    }
    // halo wave kind: 1 row below, 2 row above, 3 corners and sides
    const int hkind = interior ? 0 : (tid - NINT < 64 ? 1 : (tid - NINT < 128 ? 2 : 3));
    const bool zlo_wall = (g.lo_solid & 4) != 0, zhi_wall = (g.hi_solid & 4) != 0;
    const bool zlo_out = ((g.lo_solid | g.lo_ghost) & 4) != 0, zhi_out = ((g.hi_solid | g.hi_ghost) & 4) != 0;

    // this thread's column in tile t and the tile's z range
    struct Column {
        int gx, gy;    // grid coordinates (one outside the grid for halo columns)
        int wx, wy;    // wrapped (periodic) or clamped coordinates
        unsigned col;  // wx + nx wy
        int zs, ze;    // output planes [zs, ze)
    };
    auto column = [&](int4 sg) {
        Column c;
        const int tx = sg.x % tiles_x, ty = sg.x / tiles_x;
        c.gx = tx * TX - 1 + lx;
        c.gy = ty * TY - 1 + ly;
        c.wx = wrap_or_clamp(c.gx, nx, g.periodic & 1);
        c.wy = wrap_or_clamp(c.gy, ny, g.periodic & 2);
        c.col = (unsigned)c.wx + (unsigned)nx * (unsigned)c.wy;
        c.zs = sg.y;
        c.ze = sg.z;
        return c;
    };

    // What the next plane's build needs, loaded one plane ahead and left in
    // flight until that build starts: the stored moments (unconverted), the
    // acceleration of a force field and the plane's 1 - omega.  Converting
    // 16-bit values right after their loads, or loading 1 - omega when the
    // plane starts, would make the wave wait for its loads at that point.
    typename S::T rcur[10];
    // With FP32 storage the stored fields are loaded two plane-steps ahead,
    // into two register sets used in turn (rcur on the even steps of a
    // segment, rnx on the odd ones): one step of lookahead leaves the kernel
    // exposed to the HBM latency, which on the 512 x 256 x 256 grids
    // depends on where the buffers land in memory (up to 20 % slower launches
    // for some placements).  The 16-bit instantiations (no registers to
    // spare, compute-bound) and the walls-plus-force-field one (it would
    // spill) keep one step.
    constexpr bool kTwo = sizeof(typename S::T) == 4 && !(WALLS && FIELD);
    typename S::T rnx[kTwo ? 10 : 1];
    float gcur[3] = {0.0f, 0.0f, 0.0f};
    float ocur = p.one_minus_omega;
    auto fetch = [&](unsigned col, int zq) {
        const unsigned n = col + plane_nodes * (unsigned)zq;
        load_raw<S>(f, n, rcur);
        if constexpr (FIELD) {
#pragma unroll
            for (int a = 0; a < 3; ++a) gcur[a] = ld_at(f.g[a], n * 4u);
        }
        if (p.omo_z) ocur = p.omo_z[zq];
    };

    auto fetch_side = [&](unsigned col, int zq) {
        if constexpr (FIELD) {
            const unsigned n = col + plane_nodes * (unsigned)zq;
#pragma unroll
            for (int a = 0; a < 3; ++a) gcur[a] = ld_at(f.g[a], n * 4u);
        }
        if (p.omo_z) ocur = p.omo_z[zq];
    };

    Column c = column(t);
    if (active) {
        fetch(c.col, plane_index(c.zs - 1, nz, pz));
        if constexpr (kTwo) load_raw<S>(f, c.col + plane_nodes * (unsigned)plane_index(c.zs, nz, pz), rnx);
    }

    for (;;) {
        // the block's next segment: its first plane is loaded while the last
        // plane of this one is exchanged and gathered
        const int4 tn4 = k + 1 < p.sched_nseg ? segs[k + 1] : make_int4(-1, 0, 0, 0);
        const int tn = tn4.x;
        const Column cn = column(tn >= 0 ? tn4 : t);
        const int gx = c.gx, gy = c.gy, zs = c.zs, ze = c.ze;

        // interior column output properties
        const bool valid = interior && gx < nx && gy < ny;
        bool col_fluid = valid;
        if (valid) {
            col_fluid &= !((gx == 0) && (((g.lo_solid | g.lo_ghost) & 1)));
            col_fluid &= !((gx == nx - 1) && (((g.hi_solid | g.hi_ghost) & 1)));
            col_fluid &= !((gy == 0) && (((g.lo_solid | g.lo_ghost) & 2)));
            col_fluid &= !((gy == ny - 1) && (((g.hi_solid | g.hi_ghost) & 2)));
        }
        const int wf = (WALLS && interior) ? wall_flags(g, gx, gy) : 0;
        // Wall nodes emit nothing: their stored moments are the zero deviation
        // (rest state) and their forcing is switched off here, so every
        // population they would publish is exactly 0 and the gather needs no
        // masking.  Fluid neighbours get the bounced-back populations instead.
        bool col_solid = false;
        if (WALLS) {
            col_solid |= (c.wx == 0 && (g.lo_solid & 1)) || (c.wx == nx - 1 && (g.hi_solid & 1));
            col_solid |= (c.wy == 0 && (g.lo_solid & 2)) || (c.wy == ny - 1 && (g.hi_solid & 2));
        }
        const float gon = col_solid ? 0.0f : 1.0f;
        const float gacc[3] = {gon * p.force[0], gon * p.force[1], gon * p.force[2]};

        // The nine populations a halo column sends into the tile, unweighted
        // (D3Q27): with one velocity component fixed at s = +-1 (cy for the
        // rows below and above, cx for the corners and side columns) the
        // polynomial P(c) collapses to one in the two other components,
        // evaluated on their 3 x 3 grid.
        auto emit_halo = [&](const float A[NK], int kind, int hx, int hy) {
            float T[27];
            if (kind != 3) {
                const float s = kind == 1 ? 1.0f : -1.0f;  // cy
                eval_slice<0, 27, false>(fmaf(s, A[K010], A[K000] + A[K020]), fmaf(s, A[K110], A[K100] + A[K120]),
                                         fmaf(s, A[K011], A[K001] + A[K021]), fmaf(s, A[K210], A[K200]),
                                         fmaf(s, A[K012], A[K002]), fmaf(s, A[K111], A[K101]), A[K201], A[K102], T);
                // T[9 + 3 (cz + 1) + (cx + 1)]
                if (kind == 1) {
                    Unroll<0, 27>::run([&]<int I>() {
                        if constexpr (cy_of(I) == 1) lds[slot_of(I)][hy][hx] = T[9 + 3 * (cz_of(I) + 1) + cx_of(I) + 1];
                    });
                } else {
                    Unroll<0, 27>::run([&]<int I>() {
                        if constexpr (cy_of(I) == -1) lds[slot_of(I)][hy][hx] = T[9 + 3 * (cz_of(I) + 1) + cx_of(I) + 1];
                    });
                }
            } else {
                const float s = hx == 0 ? 1.0f : -1.0f;  // cx
                eval_slice<0, 27, false>(fmaf(s, A[K100], A[K000] + A[K200]), fmaf(s, A[K110], A[K010] + A[K210]),
                                         fmaf(s, A[K101], A[K001] + A[K201]), fmaf(s, A[K120], A[K020]),
                                         fmaf(s, A[K102], A[K002]), fmaf(s, A[K111], A[K011]), A[K021], A[K012], T);
                // T[9 + 3 (cz + 1) + (cy + 1)]
                if (hx == 0) {
                    Unroll<0, 27>::run([&]<int I>() {
                        if constexpr (cx_of(I) == 1) lds[slot_of(I)][hy][hx] = T[9 + 3 * (cz_of(I) + 1) + cy_of(I) + 1];
                    });
                } else {
                    Unroll<0, 27>::run([&]<int I>() {
                        if constexpr (cx_of(I) == -1) lds[slot_of(I)][hy][hx] = T[9 + 3 * (cz_of(I) + 1) + cy_of(I) + 1];
                    });
                }
            }
        };

        // One plane zp: build and publish its populations from the fetched
        // values, fetch the next plane (or the next tile's first plane), add
        // what arrives from plane zp to the output planes zp - 1 (aprev), zp
        // (acur) and zp + 1 (anext, which starts here), then store the
        // completed plane zp - 1.
        auto plane = [&]<int BUF>(int zp, MomentSums& aprev, MomentSums& acur, MomentSums& anext) {
            float G[27];
            if (active) {
                float m[10], gl[3];
                if constexpr (kTwo && BUF == 1)
                    convert_raw<S>(rnx, p, m);
                else
                    convert_raw<S>(rcur, p, m);
#pragma unroll
                for (int a = 0; a < 3; ++a) gl[a] = FIELD ? gon * gcur[a] : gacc[a];
                // 1 - omega with the stored Pi^neq scale folded in (see convert_raw)
                const float omo = sizeof(typename S::T) == 4 ? ocur : ocur * p.inv_scale[2];
                float A[NK];
                if (WALLS) {
                    // a wall plane (z walls) emits nothing either
                    const bool plane_solid = (zlo_wall && zp == 0) || (zhi_wall && zp == nz - 1);
                    const float gp = plane_solid ? 0.0f : 1.0f;
                    const float gz[3] = {gp * gl[0], gp * gl[1], gp * gl[2]};
                    coefficients<ORDER, LAT>(m, gz, omo, A);
                } else {
                    coefficients<ORDER, LAT>(m, gl, omo, A);
                }
                if (kDeferWeights && !interior) {
                    // a halo column only publishes what enters the tile
                    emit_halo(A, hkind, lx, ly);
                } else {
                populations<LAT, !kDeferWeights>(A, G);
                if (WALLS && TSLB_FUSED_WALLS && interior && col_fluid) {
                    // half-way bounce-back in place: a fluid node next to a wall
                    // receives its own population along -c for every c whose
                    // upstream node is solid; it holds those values right here
                    const bool zlo_adj = zlo_wall && zp == 1, zhi_adj = zhi_wall && zp == nz - 2;
                    if (wf != 0 || zlo_adj || zhi_adj) {
                        Unroll<0, 27>::run([&]<int I>() {
                            if (upstream_solid<I>(wf, zlo_adj, zhi_adj))
                                acur.template add<I>(kDeferWeights ? w216_of(I) * G[26 - I] : G[26 - I]);
                        });
                    }
                }
                Unroll<0, 27>::run([&]<int I>() {
                    if constexpr (cx_of(I) != 0 || cy_of(I) != 0) lds[slot_of(I)][ly][lx] = G[I];
                });
                }
                // the fetched values are dead once the coefficients are
                // formed: the next plane's go into the same registers and are
                // in flight across the exchange, the gather and the stores
                if constexpr (kTwo) {
                    // this step's set is free again: load the step after next
                    // into it, and the next step's force / relaxation values
                    int c2 = -1, z2 = 0;
                    if (zp + 2 <= ze) {
                        c2 = (int)c.col;
                        z2 = zp + 2;
                    } else if (tn >= 0) {
                        c2 = (int)cn.col;
                        z2 = zp + 2 == ze + 1 ? cn.zs - 1 : cn.zs;
                    }
                    if (c2 >= 0) {
                        const unsigned n2 = (unsigned)c2 + plane_nodes * (unsigned)plane_index(z2, nz, pz);
                        if constexpr (BUF == 1)
                            load_raw<S>(f, n2, rnx);
                        else
                            load_raw<S>(f, n2, rcur);
                    }
                    if (zp + 1 <= ze)
                        fetch_side(c.col, plane_index(zp + 1, nz, pz));
                    else if (tn >= 0)
                        fetch_side(cn.col, plane_index(cn.zs - 1, nz, pz));
                } else {
                if (zp + 1 <= ze)
                    fetch(c.col, plane_index(zp + 1, nz, pz));
                else if (tn >= 0)
                    fetch(cn.col, plane_index(cn.zs - 1, nz, pz));
                }
            }
            __syncthreads();
            // the 24 values arriving through LDS go to registers at once, so
            // the buffer is free again after the second barrier and the
            // stores and the next plane's build (with FP32 storage, also the
            // gather sums) form one barrier-free phase
            float F[3][3][3];  // [cz + 1][cy + 1][cx + 1]
            if (interior) {
                Unroll<0, 27>::run([&]<int I>() {
                    constexpr int X = cx_of(I), Y = cy_of(I), Z = cz_of(I);
                    if constexpr (X == 0 && Y == 0)
                        F[Z + 1][1][1] = G[I];
                    else
                        F[Z + 1][Y + 1][X + 1] = lds[slot_of(I)][ly - Y][lx - X];
                });
            }
            // With 16-bit storage the kernel is compute-bound: the sums are
            // formed before the barrier, so one wave's adds overlap the other
            // waves' LDS reads.  With FP32 storage they come after it.
            constexpr bool kSumFirst = sizeof(typename S::T) == 2;
            if constexpr (kSumFirst) {
                if (interior) {
                    add_slice<-1, false, kDeferWeights>(F[0], aprev);
                    add_slice<0, false, kDeferWeights>(F[1], acur);
                    add_slice<1, true, kDeferWeights>(F[2], anext);
                }
            }
            __syncthreads();
            if constexpr (!kSumFirst) {
                if (interior) {
                    add_slice<-1, false, kDeferWeights>(F[0], aprev);
                    add_slice<0, false, kDeferWeights>(F[1], acur);
                    add_slice<1, true, kDeferWeights>(F[2], anext);
                }
            }
            const int zo = zp - 1;
            if (interior && zo >= zs && zo < ze) {
                const bool fl = col_fluid && !(zo == 0 && zlo_out) && !(zo == nz - 1 && zhi_out);
                const bool near_wall =
                    WALLS && !TSLB_FUSED_WALLS && (wf != 0 || (zlo_wall && zo == 1) || (zhi_wall && zo == nz - 2));
                if (fl && near_wall) {
                    // next to a wall: the bounced-back populations are still
                    // missing; leave the raw sums for the fix-up pass
                    const int cc[3] = {gx, gy, zo};
                    const int fw = first_wall_face(g, cc);
                    float* side = p.wall_side + 10 * (p.wall_off[fw] + wall_layer_index(g, fw, cc));
                    side[0] = aprev.d;
#pragma unroll
                    for (int a = 0; a < 3; ++a) side[1 + a] = aprev.j[a];
#pragma unroll
                    for (int k = 0; k < 6; ++k) side[4 + k] = aprev.s[k];
                } else if (fl) {
                    float out[10];
                    if constexpr (sizeof(typename S::T) == 4)
                        finalize<LAT == 19 ? 36 : 216>(aprev, out);
                    else
                        finalize_scaled<LAT == 19 ? 36 : 216>(aprev, p.scale[0], p.scale[1], p.scale[2], out);
                    const unsigned on = (c.col + plane_nodes * (unsigned)zo) * (unsigned)sizeof(typename S::T);
#pragma unroll
                    for (int q = 0; q < 10; ++q) store_out<(MODE > 0)>(at(f.out[q], on), S::pack(out[q]));
                    if constexpr (MODE == 2) {
                        // A ghost node of an x face next to this fluid node
                        // takes its values (Section 2.3 refill; an inlet's
                        // velocity is imposed by the refill pass): stored here,
                        // into the cache line this row's stores fill anyway.
                        // This node is fluid, so that ghost lies on no other
                        // ghost face.
                        if ((g.lo_ghost & 1) && gx == 1) {
                            const unsigned og = on - (unsigned)sizeof(typename S::T);
#pragma unroll
                            for (int q = 0; q < 10; ++q) store_out<true>(at(f.out[q], og), S::pack(out[q]));
                        }
                        if ((g.hi_ghost & 1) && gx == nx - 2) {
                            const unsigned og = on + (unsigned)sizeof(typename S::T);
#pragma unroll
                            for (int q = 0; q < 10; ++q) store_out<true>(at(f.out[q], og), S::pack(out[q]));
                        }
                    }
                }
            }
        };

        // Rolling roles of the three accumulators, unrolled to their period so
        // every role is a fixed register set.
        MomentSums a0, a1, a2;
        a0.zero();
        a1.zero();
        if constexpr (kTwo) {
            // accumulator roles repeat every 3 steps, register sets every 2
            for (int zp = zs - 1; zp <= ze; zp += 6) {
                plane.template operator()<0>(zp, a0, a1, a2);
                if (zp + 1 > ze) break;
                plane.template operator()<1>(zp + 1, a1, a2, a0);
                if (zp + 2 > ze) break;
                plane.template operator()<0>(zp + 2, a2, a0, a1);
                if (zp + 3 > ze) break;
                plane.template operator()<1>(zp + 3, a0, a1, a2);
                if (zp + 4 > ze) break;
                plane.template operator()<0>(zp + 4, a1, a2, a0);
                if (zp + 5 > ze) break;
                plane.template operator()<1>(zp + 5, a2, a0, a1);
            }
            // an odd number of steps left the next segment's first plane in
            // rnx: swap the sets so that it starts on rcur again
            if (((ze - zs) & 1) != 0) {
#pragma unroll
                for (int q = 0; q < 10; ++q) {
                    const typename S::T v = rcur[q];
                    rcur[q] = rnx[q];
                    rnx[q] = v;
                }
            }
        } else {
        for (int zp = zs - 1; zp <= ze; zp += 3) {
            plane.template operator()<0>(zp, a0, a1, a2);
            if (zp + 1 > ze) break;
            plane.template operator()<0>(zp + 1, a1, a2, a0);
            if (zp + 2 > ze) break;
            plane.template operator()<0>(zp + 2, a2, a0, a1);
        }
        }
        if (tn < 0) break;
        ++k;
        t = tn4;
        c = cn;
    }
}

// Completes the fluid nodes next to a wall after the tiled update: adds the
// half-way bounce-back populations (the node's own post-collision population
// along -c, arriving along c for every c whose upstream node is a wall) to
// the raw sums the update left in the side buffer, then finalises and
// stores.  Threads enumerate the layers next to each wall face; a node next
// to several walls is done once, by its first wall face.
template <class S, int ORDER, int LAT>
__global__ void __launch_bounds__(256) wall_fixup_kernel(const FieldPtrs<typename S::T> f, StepParams p,
                                                         long long total) {
    const Geometry& g = p.geo;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= total) return;
    int fw = -1;
    long long local = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (p.wall_off[k] >= 0 && tid >= p.wall_off[k]) {
            fw = k;
            local = tid - p.wall_off[k];
        }
    }
    if (fw < 0) return;
    const int d = fw >> 1, d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    if (local >= (long long)g.n[d1] * g.n[d2]) return;
    int c[3];
    c[d] = (fw & 1) ? g.n[d] - 2 : 1;
    c[d1] = (int)(local % g.n[d1]);
    c[d2] = (int)(local / g.n[d1]);
    if (!is_fluid(g, c[0], c[1], c[2]) || first_wall_face(g, c) != fw) return;

    const unsigned node = (unsigned)c[0] + (unsigned)g.n[0] * ((unsigned)c[1] + (unsigned)g.n[1] * (unsigned)c[2]);
    float m[10], gg[3];
    load_node<S>(f, node, p, m);
#pragma unroll
    for (int a = 0; a < 3; ++a) gg[a] = f.g[a] ? ld_at(f.g[a], node * 4u) : p.force[a];
    float A[NK], G[27];
    coefficients<ORDER, LAT>(m, gg, omo_at(p, c[2]), A);
    populations<LAT>(A, G);

    const float* side = p.wall_side + 10 * local + 10 * p.wall_off[fw];
    MomentSums a;
    a.d = side[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) a.j[k] = side[1 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) a.s[k] = side[4 + k];
    const int wf = wall_flags(g, c[0], c[1]);
    const bool zlo = (g.lo_solid & 4) && c[2] == 1, zhi = (g.hi_solid & 4) && c[2] == g.n[2] - 2;
    Unroll<0, 27>::run([&]<int I>() {
        if (upstream_solid<I>(wf, zlo, zhi)) a.template add<I>(G[26 - I]);
    });
    float out[10];
    finalize<LAT == 19 ? 36 : 216>(a, out);
    const unsigned on = node * (unsigned)sizeof(typename S::T);
    *at(f.out[0], on) = S::store(out[0], p.scale[0]);
#pragma unroll
    for (int q = 1; q < 4; ++q) *at(f.out[q], on) = S::store(out[q], p.scale[1]);
#pragma unroll
    for (int q = 4; q < 10; ++q) *at(f.out[q], on) = S::store(out[q], p.scale[2]);
}

template <class S>
bool rows_whole_lines(const StepParams& p) {
    return ((long long)p.geo.n[0] * (long long)sizeof(typename S::T)) % 128 == 0;
}
inline bool x_ghost_faces(const StepParams& p) { return ((p.geo.lo_ghost | p.geo.hi_ghost) & 1) != 0; }

template <class S, bool WALLS, bool FIELD, int ORDER, int LAT>
hipError_t launch_t(const void* in, void* out, const StepParams& p, hipStream_t s) {
    const int tiles_x = (p.geo.n[0] + TX - 1) / TX;
    if (p.geo.N >= (1LL << 30)) return hipErrorInvalidValue;  // 32-bit node offsets
    if (!p.sched || p.sched_grid < 8 || p.sched_nseg < 1) return hipErrorInvalidValue;
    const FieldPtrs<typename S::T> f = field_ptrs<S>(in, out, p);
    // non-temporal output stores only when every row starts on a cache line
    const bool nt = rows_whole_lines<S>(p);
    const dim3 grid(p.sched_grid), block(NTHREADS);
    if constexpr (!WALLS && !FIELD) {
        if (nt && x_ghost_faces(p)) {
            hipLaunchKernelGGL((update_tiled_kernel<S, false, false, ORDER, LAT, 2>), grid, block, 0, s, f, p, tiles_x);
            return hipGetLastError();
        }
    }
    if (nt)
        hipLaunchKernelGGL((update_tiled_kernel<S, WALLS, FIELD, ORDER, LAT, 1>), grid, block, 0, s, f, p, tiles_x);
    else
        hipLaunchKernelGGL((update_tiled_kernel<S, WALLS, FIELD, ORDER, LAT, 0>), grid, block, 0, s, f, p, tiles_x);
    return hipGetLastError();
}

template <class S, int ORDER, int LAT>
hipError_t launch_o(const void* in, void* out, const StepParams& p, hipStream_t s) {
    const bool walls = (p.geo.lo_solid | p.geo.hi_solid) != 0;
    const bool field = p.gfield != nullptr;
    if (walls)
        return field ? launch_t<S, true, true, ORDER, LAT>(in, out, p, s)
                     : launch_t<S, true, false, ORDER, LAT>(in, out, p, s);
    return field ? launch_t<S, false, true, ORDER, LAT>(in, out, p, s)
                 : launch_t<S, false, false, ORDER, LAT>(in, out, p, s);
}

template <class S, int LAT>
hipError_t launch_l(const void* in, void* out, const StepParams& p, hipStream_t s) {
    return p.order == 2 ? launch_o<S, 2, LAT>(in, out, p, s) : launch_o<S, 3, LAT>(in, out, p, s);
}

template <class S>
hipError_t launch_s(const void* in, void* out, const StepParams& p, hipStream_t s) {
    return p.lattice == 19 ? launch_l<S, 19>(in, out, p, s) : launch_l<S, 27>(in, out, p, s);
}

}  // namespace

template <class S>
hipError_t fixup_s(const void* in, void* out, const StepParams& p, hipStream_t s) {
    if (TSLB_FUSED_WALLS || p.wall_nodes == 0) return hipSuccess;  // the update did the bounce-back
    const FieldPtrs<typename S::T> f = field_ptrs<S>(in, out, p);
    const int block = 256;
    const unsigned grid = (unsigned)((p.wall_nodes + block - 1) / block);
    if (p.lattice == 19) {
        if (p.order == 2)
            hipLaunchKernelGGL((wall_fixup_kernel<S, 2, 19>), dim3(grid), dim3(block), 0, s, f, p, p.wall_nodes);
        else
            hipLaunchKernelGGL((wall_fixup_kernel<S, 3, 19>), dim3(grid), dim3(block), 0, s, f, p, p.wall_nodes);
    } else if (p.order == 2) {
        hipLaunchKernelGGL((wall_fixup_kernel<S, 2, 27>), dim3(grid), dim3(block), 0, s, f, p, p.wall_nodes);
    } else {
        hipLaunchKernelGGL((wall_fixup_kernel<S, 3, 27>), dim3(grid), dim3(block), 0, s, f, p, p.wall_nodes);
    }
    return hipGetLastError();
}

bool tiled_uses_wall_side() { return TSLB_FUSED_WALLS == 0; }

hipError_t tiled_schedule(const Geometry& g, std::vector<int4>& seg, int& grid, int& nseg) {
    const int columns = ((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY);
    const int resident = (compute_units() * kBlocksPerCu + 7) & ~7;
    Schedule s = build_schedule(columns, g.n[2], resident);
    if (s.grid < 8 || s.nseg < 1) return hipErrorInvalidValue;
    seg = std::move(s.seg);
    grid = s.grid;
    nseg = s.nseg;
    return hipSuccess;
}

bool tiled_writes_x_ghosts(int storage, const StepParams& p) {
    const bool walls = (p.geo.lo_solid | p.geo.hi_solid) != 0;
    const bool nt = storage == 0 ? rows_whole_lines<StoreF32>(p) : rows_whole_lines<StoreF16>(p);
    return !walls && p.gfield == nullptr && nt && x_ghost_faces(p);
}

hipError_t launch_wall_fixup(int storage, const void* in, void* out, const StepParams& p, hipStream_t s) {
    switch (storage) {
    case 0: return fixup_s<StoreF32>(in, out, p, s);
    case 1: return fixup_s<StoreF16>(in, out, p, s);
    case 2: return fixup_s<StoreBF16>(in, out, p, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_update_tiled(int storage, const void* in, void* out, const StepParams& p, hipStream_t s) {
    switch (storage) {
    case 0: return launch_s<StoreF32>(in, out, p, s);
    case 1: return launch_s<StoreF16>(in, out, p, s);
    case 2: return launch_s<StoreBF16>(in, out, p, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace tslb
