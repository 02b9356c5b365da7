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
// Block = TX x TY interior columns plus a one-node halo ring (extra waves);
// it marches tz planes (plus one halo plane each side), tz chosen per grid
// at launch.  A plane's emitted
// populations with (cx, cy) != (0, 0) go through LDS; the three with
// cx = cy = 0 stay in the thread.  Contributions to the output planes
// p - 1, p, p + 1 are accumulated in three rolling register sets.
#include "tslb_tiles.h"

namespace tslb {
namespace {

using namespace tile;


template <class S, bool WALLS, bool FIELD, int ORDER, int LAT>
__global__ void __launch_bounds__(NTHREADS, TSLB_WAVES_PER_EU) update_tiled_kernel(const FieldPtrs<typename S::T> f, StepParams p,
                                                                   int tiles_x, int tiles_y, int tiles_z, int TZ) {
    __shared__ float lds_all[NBUF][NSLOT][LY][LX];
    const Geometry& g = p.geo;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned plane_nodes = (unsigned)nx * (unsigned)ny;

    // Tile order: consecutive block ids are dealt round-robin to the 8 XCDs;
    // give each XCD a contiguous run of tiles, x fastest, then y, then z, so
    // the tiles that run together on one XCD are x and y neighbours marching
    // the same planes: the halo columns and rows they read from each other
    // are then L2 hits instead of HBM reads.
    const int b = xcd_tile(blockIdx.x, tiles_x * tiles_y * tiles_z);
    if (b < 0) return;  // padding block (before any barrier)
    const int tx = b % tiles_x;
    const int ty = (b / tiles_x) % tiles_y;
    const int tz = b / (tiles_x * tiles_y);
    const int x0 = tx * TX, y0 = ty * TY;
    const int zs = tz * TZ;
    const int ze = min(zs + TZ, nz);

    // thread -> LDS column (lx, ly); interior columns first, whole waves
    const int tid = threadIdx.x;
    int lx, ly;
    bool active = true;
    const bool interior = tid < NINT;
    if (interior) {
        lx = 1 + tid % TX;
        ly = 1 + tid / TX;
    } else {
        const int h = tid - NINT;
        if (h < LX) {
            lx = h;
            ly = 0;
        } else if (h < 2 * LX) {
            lx = h - LX;
            ly = LY - 1;
        } else if (h < 2 * LX + 2 * TY) {
            const int k = h - 2 * LX;
            lx = (k < TY) ? 0 : LX - 1;
            ly = 1 + (k % TY);
        } else {
            lx = 0;
            ly = 0;
            active = false;
        }
    }
    const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
    const int wx = wrap_or_clamp(gx, nx, g.periodic & 1);
    const int wy = wrap_or_clamp(gy, ny, g.periodic & 2);
    const unsigned col = (unsigned)wx + (unsigned)nx * (unsigned)wy;
    const bool pz = (g.periodic & 4) != 0;

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
        col_solid |= (wx == 0 && (g.lo_solid & 1)) || (wx == nx - 1 && (g.hi_solid & 1));
        col_solid |= (wy == 0 && (g.lo_solid & 2)) || (wy == ny - 1 && (g.hi_solid & 2));
    }
    const bool zlo_wall = (g.lo_solid & 4) != 0, zhi_wall = (g.hi_solid & 4) != 0;
    const bool zlo_out = ((g.lo_solid | g.lo_ghost) & 4) != 0, zhi_out = ((g.hi_solid | g.hi_ghost) & 4) != 0;

    const float gon = col_solid ? 0.0f : 1.0f;
    float gacc[3] = {gon * p.force[0], gon * p.force[1], gon * p.force[2]};

    float mcur[10];
    if (active) load_node<S>(f, col + plane_nodes * (unsigned)plane_index(zs - 1, nz, pz), p, mcur);
    // With a prefetch depth of 2 the moments of plane zp + 1 are already in
    // registers (m_ahead) while plane zp is processed, and the loads of plane
    // zp + 2 are issued: twice the bytes in flight per thread.
    float m_ahead[10];
    if (TSLB_PREFETCH_DEPTH == 2 && active)
        load_node<S>(f, col + plane_nodes * (unsigned)plane_index(zs, nz, pz), p, m_ahead);

    // Finalised moments of one output node, stored at byte offset pend_on.
    constexpr bool kDefer = TSLB_DEFER_STORE < 0 ? WALLS : TSLB_DEFER_STORE != 0;
    float pend[10];
    unsigned pend_on = 0;
    bool pend_valid = false;
    auto store_pending = [&]() {
        if (!pend_valid) return;
        store_out(at(f.out[0], pend_on), S::store(pend[0], p.scale[0]));
#pragma unroll
        for (int q = 1; q < 4; ++q) store_out(at(f.out[q], pend_on), S::store(pend[q], p.scale[1]));
#pragma unroll
        for (int q = 4; q < 10; ++q) store_out(at(f.out[q], pend_on), S::store(pend[q], p.scale[2]));
        pend_valid = false;
    };

    // One plane zp with moments mcur: prefetch the next plane into mnext,
    // build and publish this plane's populations, add what arrives from it
    // to the output planes zp - 1 (aprev), zp (acur) and zp + 1 (anext, which
    // starts here), then store the completed plane zp - 1.
    auto plane = [&](int zp, MomentSums& aprev, MomentSums& acur, MomentSums& anext) {
        const unsigned node = col + plane_nodes * (unsigned)plane_index(zp, nz, pz);
        float(&lds)[NSLOT][LY][LX] = lds_all[NBUF == 2 ? ((zp - zs + 1) & 1) : 0];
        float mnext[10];
        const bool have_next = zp + 1 <= ze;
        if (TSLB_PREFETCH_DEPTH == 1 && TSLB_EARLY_PREFETCH && active && have_next)
            load_node<S>(f, col + plane_nodes * (unsigned)plane_index(zp + 1, nz, pz), p, mnext);

        float G[27];
        if (active) {
            if (FIELD) {
#pragma unroll
                for (int a = 0; a < 3; ++a) gacc[a] = gon * ld_at(f.g[a], node * 4u);
            }
            float A[NK];
            const float omo = omo_at(p, plane_index(zp, nz, pz));
            if (WALLS) {
                // a wall plane (z walls) emits nothing either
                const bool plane_solid = (zlo_wall && zp == 0) || (zhi_wall && zp == nz - 1);
                const float gp = plane_solid ? 0.0f : 1.0f;
                const float gz[3] = {gp * gacc[0], gp * gacc[1], gp * gacc[2]};
                coefficients<ORDER, LAT>(mcur, gz, omo, A);
            } else {
                coefficients<ORDER, LAT>(mcur, gacc, omo, A);
            }
            populations<LAT>(A, G);
            if (WALLS && TSLB_FUSED_WALLS && interior && col_fluid) {
                // half-way bounce-back in place: a fluid node next to a wall
                // receives its own population along -c for every c whose
                // upstream node is solid; it holds those values right here
                const bool zlo_adj = zlo_wall && zp == 1, zhi_adj = zhi_wall && zp == nz - 2;
                if (wf != 0 || zlo_adj || zhi_adj) {
                    Unroll<0, 27>::run([&]<int I>() {
                        if (upstream_solid<I>(wf, zlo_adj, zhi_adj)) acur.template add<I>(G[26 - I]);
                    });
                }
            }
            Unroll<0, 27>::run([&]<int I>() {
                if constexpr (cx_of(I) != 0 || cy_of(I) != 0) lds[slot_of(I)][ly][lx] = G[I];
            });
            // the previous plane's outputs go out while this plane is built
            if (kDefer) store_pending();
            // prefetch the next plane once this plane's moments are consumed;
            // the loads are in flight across the exchange and the gather
            // (mcur is dead once the coefficients are formed, so the next
            // plane's moments go straight into it: no register copies)
            if (TSLB_PREFETCH_DEPTH == 1 && !TSLB_EARLY_PREFETCH && have_next)
                load_node<S>(f, col + plane_nodes * (unsigned)plane_index(zp + 1, nz, pz), p, mcur);
            if (TSLB_PREFETCH_DEPTH == 2 && zp + 2 <= ze)
                load_node<S>(f, col + plane_nodes * (unsigned)plane_index(zp + 2, nz, pz), p, mnext);
        }
        __syncthreads();
        // gather the populations arriving from this plane, one cz slice at a
        // time (nine values), and reduce each slice straight into its plane
        auto gather_slice = [&]<int CZ>(float (&F)[3][3]) {
            Unroll<0, 9>::run([&]<int K>() {
                constexpr int I = 9 * (CZ + 1) + K;
                constexpr int X = cx_of(I), Y = cy_of(I);
                if constexpr (X == 0 && Y == 0)
                    F[Y + 1][X + 1] = G[I];
                else
                    F[Y + 1][X + 1] = lds[slot_of(I)][ly - Y][lx - X];
            });
        };
        constexpr bool kEarly = TSLB_EARLY_RELEASE && NBUF == 1;
        if constexpr (kEarly) {
            float F3[3][3][3];
            if (interior) {
                gather_slice.template operator()<-1>(F3[0]);
                gather_slice.template operator()<0>(F3[1]);
                gather_slice.template operator()<1>(F3[2]);
            }
            __syncthreads();  // the buffer is free for the next plane
            if (interior) {
                add_slice<-1>(F3[0], aprev);
                add_slice<0>(F3[1], acur);
                add_slice<1, true>(F3[2], anext);
            }
        } else if (interior) {
            float F[3][3];
            gather_slice.template operator()<-1>(F);
            add_slice<-1>(F, aprev);
            gather_slice.template operator()<0>(F);
            add_slice<0>(F, acur);
            gather_slice.template operator()<1>(F);
            add_slice<1, true>(F, anext);
        }
        const int zo = zp - 1;
        if (interior && zo >= zs && zo < ze) {
            const bool fl = col_fluid && !(zo == 0 && zlo_out) && !(zo == nz - 1 && zhi_out);
            const bool near_wall =
                WALLS && !TSLB_FUSED_WALLS && (wf != 0 || (zlo_wall && zo == 1) || (zhi_wall && zo == nz - 2));
            if (fl && near_wall) {
                // next to a wall: the bounced-back populations are still missing;
                // leave the raw sums for the fix-up pass
                const int c[3] = {gx, gy, zo};
                const int fw = first_wall_face(g, c);
                float* side = p.wall_side + 10 * (p.wall_off[fw] + wall_layer_index(g, fw, c));
                side[0] = aprev.d;
#pragma unroll
                for (int a = 0; a < 3; ++a) side[1 + a] = aprev.j[a];
#pragma unroll
                for (int k = 0; k < 6; ++k) side[4 + k] = aprev.s[k];
            } else if (fl) {
                finalize<LAT == 19 ? 36 : 216>(aprev, pend);
                pend_on = (col + plane_nodes * (unsigned)zo) * (unsigned)sizeof(typename S::T);
                pend_valid = true;
                if (!kDefer) store_pending();
            }
        }
        if (TSLB_PREFETCH_DEPTH == 2) {
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                mcur[q] = m_ahead[q];
                m_ahead[q] = mnext[q];
            }
        } else if (TSLB_EARLY_PREFETCH && have_next) {
#pragma unroll
            for (int q = 0; q < 10; ++q) mcur[q] = mnext[q];
        }
        if (NBUF == 1 && !kEarly) __syncthreads();
    };

    // Rolling roles of the three accumulators, unrolled to their period so
    // every role is a fixed register set.
    MomentSums a0, a1, a2;
    a0.zero();
    a1.zero();
    for (int zp = zs - 1; zp <= ze; zp += 3) {
        plane(zp, a0, a1, a2);
        if (zp + 1 > ze) break;
        plane(zp + 1, a1, a2, a0);
        if (zp + 2 > ze) break;
        plane(zp + 2, a2, a0, a1);
    }
    store_pending();
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

template <class S, bool WALLS, bool FIELD, int ORDER, int LAT>
hipError_t launch_t(const void* in, void* out, const StepParams& p, hipStream_t s) {
    const int tiles_x = (p.geo.n[0] + TX - 1) / TX;
    const int tiles_y = (p.geo.n[1] + TY - 1) / TY;
    const int TZ = choose_tz(tiles_x * tiles_y, p.geo.n[2], compute_units() * kBlocksPerCu);
    const int tiles_z = (p.geo.n[2] + TZ - 1) / TZ;
    const unsigned nblk = (unsigned)tiles_x * tiles_y * tiles_z;
    if (p.geo.N >= (1LL << 30)) return hipErrorInvalidValue;  // 32-bit node offsets
    const FieldPtrs<typename S::T> f = field_ptrs<S>(in, out, p);
    hipLaunchKernelGGL((update_tiled_kernel<S, WALLS, FIELD, ORDER, LAT>), dim3(xcd_grid(nblk)), dim3(NTHREADS), 0, s, f, p, tiles_x,
                       tiles_y, tiles_z, TZ);
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
