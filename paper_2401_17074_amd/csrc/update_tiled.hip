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
#include "tslb_internal.h"

namespace tslb {
namespace {

#ifndef TSLB_TILE_X
#define TSLB_TILE_X 64
#endif
#ifndef TSLB_TILE_Y
#define TSLB_TILE_Y 12
#endif
#ifndef TSLB_NT_STORE
#define TSLB_NT_STORE 1
#endif
#ifndef TSLB_WAVES_PER_EU
#define TSLB_WAVES_PER_EU 4
#endif
constexpr int TX = TSLB_TILE_X;              // interior tile width (64: one wave per row)
constexpr int TY = TSLB_TILE_Y;              // interior rows
constexpr int LX = TX + 2, LY = TY + 2;      // LDS tile with halo
constexpr int NINT = TX * TY;                // interior threads (whole waves)
constexpr int NHALO = 2 * LX + 2 * TY;       // halo columns
constexpr int NTHREADS = NINT + ((NHALO + 63) / 64) * 64;
constexpr int NSLOT = 24;                    // populations with (cx, cy) != (0, 0)

__host__ __device__ constexpr int slot_of(int I) { return I - (I > 4) - (I > 13) - (I > 22); }

// monomial coefficient indices: K<ex><ey><ez> multiplies cx^ex cy^ey cz^ez
enum {
    K000, K100, K010, K001, K200, K020, K002, K110, K101, K011,
    K210, K201, K120, K021, K102, K012, K111, NK
};

// Coefficients of P(c) = sum_k A_k m_k(c) for a node with moments m
// (drho, u, Pi) and acceleration g; omo = 1 - omega (see tslb_device.h for
// P).  Equilibrium part from expanding rho [3 cu + 9/2 cu^2 - 3/2 u^2 +
// 9/2 cu^3 - 9/2 cu u^2] with c_a^3 = c_a; non-equilibrium part from
// (1 - omega) [9/2 cPc - 3/2 tr Pi + 27/2 cPc cu - 9/2 tr Pi cu - 9 c.Pi u].
__device__ __forceinline__ void coefficients(const float m[10], const float g[3], float omo, float A[NK]) {
    const float dr = m[0], rho = 1.0f + dr;
    const float ux = m[1], uy = m[2], uz = m[3];
    const float pxx = omo * m[4], pyy = omo * m[5], pzz = omo * m[6];
    const float pxy = omo * m[7], pxz = omo * m[8], pyz = omo * m[9];
    const float rx = rho * ux, ry = rho * uy, rz = rho * uz;
    const float uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
    const float u2 = uxx + uyy + uzz;
    const float tr = pxx + pyy + pzz;
    A[K000] = dr - 1.5f * (rho * u2 + tr);
    A[K200] = 4.5f * (rx * ux + pxx);
    A[K020] = 4.5f * (ry * uy + pyy);
    A[K002] = 4.5f * (rz * uz + pzz);
    A[K110] = 9.0f * (rx * uy + pxy);
    A[K101] = 9.0f * (rx * uz + pxz);
    A[K011] = 9.0f * (ry * uz + pyz);
    const float base = 3.0f - 4.5f * u2;
    const float pux = pxx * ux + pxy * uy + pxz * uz;
    const float puy = pxy * ux + pyy * uy + pyz * uz;
    const float puz = pxz * ux + pyz * uy + pzz * uz;
    const float t45 = 4.5f * tr;
    A[K100] = rx * (base + 4.5f * uxx) + ux * (13.5f * pxx - t45) - 9.0f * pux + 3.0f * rho * g[0];
    A[K010] = ry * (base + 4.5f * uyy) + uy * (13.5f * pyy - t45) - 9.0f * puy + 3.0f * rho * g[1];
    A[K001] = rz * (base + 4.5f * uzz) + uz * (13.5f * pzz - t45) - 9.0f * puz + 3.0f * rho * g[2];
    A[K210] = 13.5f * (rx * ux * uy + pxx * uy + 2.0f * pxy * ux);
    A[K201] = 13.5f * (rx * ux * uz + pxx * uz + 2.0f * pxz * ux);
    A[K120] = 13.5f * (ry * uy * ux + pyy * ux + 2.0f * pxy * uy);
    A[K021] = 13.5f * (ry * uy * uz + pyy * uz + 2.0f * pyz * uy);
    A[K102] = 13.5f * (rz * uz * ux + pzz * ux + 2.0f * pxz * uz);
    A[K012] = 13.5f * (rz * uz * uy + pzz * uy + 2.0f * pyz * uz);
    A[K111] = 27.0f * (rx * uy * uz + pxy * uz + pxz * uy + pyz * ux);
}

// Values of the 2D polynomial Q(cx, cy) = sum b_ab cx^a cy^b on the 3 x 3
// velocity grid of one cz slice, written to G[base + 3 (cy + 1) + (cx + 1)]
// with the exact weight factor 4^n0 applied.
template <int CZ>
__device__ __forceinline__ void eval_slice(float b00, float b10, float b01, float b20, float b02, float b11, float b21,
                                           float b12, float G[27]) {
    // along x for each power of cy
    const float s0 = b00 + b20, s1 = b01 + b21;
    const float r0[3] = {s0 - b10, b00, s0 + b10};
    const float r1[3] = {s1 - b11, b01, s1 + b11};
    const float r2[3] = {b02 - b12, b02, b02 + b12};
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) {
        const float t = r0[ix] + r2[ix];
        const float q[3] = {t - r1[ix], r0[ix], t + r1[ix]};
#pragma unroll
        for (int iy = 0; iy < 3; ++iy) {
            const int I = 9 * (CZ + 1) + 3 * iy + ix;
            const float w = (float)(1 << (2 * ((ix == 1) + (iy == 1) + (CZ == 0))));
            G[I] = (w == 1.0f) ? q[iy] : w * q[iy];
        }
    }
}

__device__ __forceinline__ void populations(const float A[NK], float G[27]) {
    eval_slice<0>(A[K000], A[K100], A[K010], A[K200], A[K020], A[K110], A[K210], A[K120], G);
    const float e00 = A[K000] + A[K002], e10 = A[K100] + A[K102], e01 = A[K010] + A[K012];
    eval_slice<1>(e00 + A[K001], e10 + A[K101], e01 + A[K011], A[K200] + A[K201], A[K020] + A[K021],
                  A[K110] + A[K111], A[K210], A[K120], G);
    eval_slice<-1>(e00 - A[K001], e10 - A[K101], e01 - A[K011], A[K200] - A[K201], A[K020] - A[K021],
                   A[K110] - A[K111], A[K210], A[K120], G);
}

// Moments of one arriving cz slice F[cy+1][cx+1], added to the output plane
// accumulator: sum F, sum F c and sum F c c with c = (cx, cy, CZ).
template <int CZ, bool ASSIGN = false>
__device__ __forceinline__ void add_slice(const float F[3][3], MomentSums& a) {
    float s[3], d[3], t[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        s[r] = F[r][0] + F[r][2];
        d[r] = F[r][2] - F[r][0];
        t[r] = s[r] + F[r][1];
    }
    const float m02 = t[2] + t[0];
    const float m00 = m02 + t[1];
    const float m01 = t[2] - t[0];
    const float m10 = d[0] + d[1] + d[2];
    const float m11 = d[2] - d[0];
    const float m20 = s[0] + s[1] + s[2];
    if constexpr (ASSIGN) {
        // first contribution to a fresh output plane (only the CZ != 0 slices
        // touch all ten sums)
        static_assert(CZ != 0, "assignment needs a slice that covers every moment");
        a.d = m00;
        a.j[0] = m10;
        a.j[1] = m01;
        a.s[0] = m20;
        a.s[1] = m02;
        a.s[3] = m11;
        a.j[2] = CZ * m00;
        a.s[2] = m00;
        a.s[4] = CZ * m10;
        a.s[5] = CZ * m01;
    } else {
        a.d += m00;
        a.j[0] += m10;
        a.j[1] += m01;
        a.s[0] += m20;
        a.s[1] += m02;
        a.s[3] += m11;
        if (CZ != 0) {
            a.j[2] += CZ * m00;
            a.s[2] += m00;
            a.s[4] += CZ * m10;
            a.s[5] += CZ * m01;
        }
    }
}

// Output stores: the new level is not read again by this launch, so it may
// bypass L2 allocation (non-temporal) and leave the cache to the halo reads.
template <class T>
__device__ __forceinline__ void store_out(T* p, T v) {
    if constexpr (TSLB_NT_STORE) {
        if constexpr (sizeof(T) == 4)
            __builtin_nontemporal_store(__builtin_bit_cast(float, v), reinterpret_cast<float*>(p));
        else
            __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), reinterpret_cast<unsigned short*>(p));
    } else {
        *p = v;
    }
}

// Field q of node n: a uniform per-field base plus a 32-bit node offset, so
// the address is one scalar base and one shared vector offset (the grid
// holds fewer than 2^30 nodes, checked at launch).
template <class T>
__device__ __forceinline__ T ld_at(const T* __restrict__ base, unsigned byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <class T>
__device__ __forceinline__ T* at(T* base, unsigned byte_off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}

// Per-field base pointers, passed as kernel arguments so each one sits in
// scalar registers and every access is that base plus one shared 32-bit
// vector offset (no per-field 64-bit address arithmetic).
template <class T>
struct FieldPtrs {
    const T* in[10];
    T* out[10];
    const float* g[3];
};

template <class S>
__device__ __forceinline__ void load_node(const FieldPtrs<typename S::T>& f, unsigned n, const StepParams& p,
                                          float m[10]) {
    const unsigned off = n * (unsigned)sizeof(typename S::T);
    m[0] = S::load(ld_at(f.in[0], off), p.inv_scale[0]);
#pragma unroll
    for (int q = 1; q < 4; ++q) m[q] = S::load(ld_at(f.in[q], off), p.inv_scale[1]);
#pragma unroll
    for (int q = 4; q < 10; ++q) m[q] = S::load(ld_at(f.in[q], off), p.inv_scale[2]);
}

// Plane index of zp in [-1, nz]: one wrap for a periodic axis, else clamp.
__device__ __forceinline__ int plane_index(int zp, int nz, bool periodic) {
    if (periodic) return zp < 0 ? zp + nz : (zp >= nz ? zp - nz : zp);
    return zp < 0 ? 0 : (zp >= nz ? nz - 1 : zp);
}

// In-range index of coordinate v on an axis of n nodes: periodic axes wrap
// (any v, so lanes of a tile wider than the grid stay in bounds), others clamp
// (clamped values are never used by a fluid node).
__device__ __forceinline__ int wrap_or_clamp(int v, int n, bool periodic) {
    if (periodic) {
        v %= n;
        return v < 0 ? v + n : v;
    }
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// Per-lane wall flags of an interior column: bit 0 lo-x, 1 hi-x, 2 lo-y,
// 3 hi-y set when the neighbour on that side is a wall node.
__device__ __forceinline__ int wall_flags(const Geometry& g, int gx, int gy) {
    int f = 0;
    f |= ((g.lo_solid & 1) && gx == 1) ? 1 : 0;
    f |= ((g.hi_solid & 1) && gx == g.n[0] - 2) ? 2 : 0;
    f |= ((g.lo_solid & 2) && gy == 1) ? 4 : 0;
    f |= ((g.hi_solid & 2) && gy == g.n[1] - 2) ? 8 : 0;
    return f;
}

// Is the upstream node of direction I solid, for an output node with
// in-plane flags wf and z flags zlo (plane below is a wall) / zhi?
template <int I>
__device__ __forceinline__ bool upstream_solid(int wf, bool zlo, bool zhi) {
    constexpr int X = cx_of(I), Y = cy_of(I), Z = cz_of(I);
    bool s = false;
    if (X == 1) s |= (wf & 1) != 0;
    if (X == -1) s |= (wf & 2) != 0;
    if (Y == 1) s |= (wf & 4) != 0;
    if (Y == -1) s |= (wf & 8) != 0;
    if (Z == 1) s |= zlo;
    if (Z == -1) s |= zhi;
    return s;
}

template <class S, bool WALLS, bool FIELD>
__global__ void __launch_bounds__(NTHREADS, TSLB_WAVES_PER_EU) update_tiled_kernel(const FieldPtrs<typename S::T> f, StepParams p,
                                                                   int tiles_x, int tiles_y, int tiles_z, int TZ) {
    __shared__ float lds[NSLOT][LY][LX];
    const Geometry& g = p.geo;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned plane_nodes = (unsigned)nx * (unsigned)ny;

    // Tile order: consecutive block ids are dealt round-robin to the 8 XCDs;
    // give each XCD a contiguous run of tiles, x fastest, then y, then z, so
    // the tiles that run together on one XCD are x and y neighbours marching
    // the same planes: the halo columns and rows they read from each other
    // are then L2 hits instead of HBM reads.
    const int nblk = tiles_x * tiles_y * tiles_z;
    int b = blockIdx.x;
    if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
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

    // One plane zp with moments mcur: prefetch the next plane into mnext,
    // build and publish this plane's populations, add what arrives from it
    // to the output planes zp - 1 (aprev), zp (acur) and zp + 1 (anext, which
    // starts here), then store the completed plane zp - 1.
    auto plane = [&](int zp, MomentSums& aprev, MomentSums& acur, MomentSums& anext) {
        const unsigned node = col + plane_nodes * (unsigned)plane_index(zp, nz, pz);
        float mnext[10];
        const bool have_next = zp + 1 <= ze;

        float G[27];
        if (active) {
            if (FIELD) {
#pragma unroll
                for (int a = 0; a < 3; ++a) gacc[a] = gon * ld_at(f.g[a], node * 4u);
            }
            float A[NK];
            if (WALLS) {
                // a wall plane (z walls) emits nothing either
                const bool plane_solid = (zlo_wall && zp == 0) || (zhi_wall && zp == nz - 1);
                const float gp = plane_solid ? 0.0f : 1.0f;
                const float gz[3] = {gp * gacc[0], gp * gacc[1], gp * gacc[2]};
                coefficients(mcur, gz, p.one_minus_omega, A);
            } else {
                coefficients(mcur, gacc, p.one_minus_omega, A);
            }
            populations(A, G);
            Unroll<0, 27>::run([&]<int I>() {
                if constexpr (cx_of(I) != 0 || cy_of(I) != 0) lds[slot_of(I)][ly][lx] = G[I];
            });
            // prefetch the next plane once this plane's moments are consumed;
            // the loads are in flight across the exchange and the gather
            if (have_next) load_node<S>(f, col + plane_nodes * (unsigned)plane_index(zp + 1, nz, pz), p, mnext);
        }
        __syncthreads();
        if (interior) {
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
            const bool near_wall = WALLS && (wf != 0 || (zlo_wall && zo == 1) || (zhi_wall && zo == nz - 2));
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
                float m[10];
                finalize(aprev, m);
                const unsigned on = (col + plane_nodes * (unsigned)zo) * (unsigned)sizeof(typename S::T);
                store_out(at(f.out[0], on), S::store(m[0], p.scale[0]));
#pragma unroll
                for (int q = 1; q < 4; ++q) store_out(at(f.out[q], on), S::store(m[q], p.scale[1]));
#pragma unroll
                for (int q = 4; q < 10; ++q) store_out(at(f.out[q], on), S::store(m[q], p.scale[2]));
            }
        }
        if (have_next) {
#pragma unroll
            for (int q = 0; q < 10; ++q) mcur[q] = mnext[q];
        }
        __syncthreads();
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
}

// Completes the fluid nodes next to a wall after the tiled update: adds the
// half-way bounce-back populations (the node's own post-collision population
// along -c, arriving along c for every c whose upstream node is a wall) to
// the raw sums the update left in the side buffer, then finalises and
// stores.  Threads enumerate the layers next to each wall face; a node next
// to several walls is done once, by its first wall face.
template <class S>
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
    coefficients(m, gg, p.one_minus_omega, A);
    populations(A, G);

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
    finalize(a, out);
    const unsigned on = node * (unsigned)sizeof(typename S::T);
    *at(f.out[0], on) = S::store(out[0], p.scale[0]);
#pragma unroll
    for (int q = 1; q < 4; ++q) *at(f.out[q], on) = S::store(out[q], p.scale[1]);
#pragma unroll
    for (int q = 4; q < 10; ++q) *at(f.out[q], on) = S::store(out[q], p.scale[2]);
}

template <class S>
FieldPtrs<typename S::T> field_ptrs(const void* in, void* out, const StepParams& p) {
    using T = typename S::T;
    FieldPtrs<T> f;
    for (int q = 0; q < 10; ++q) {
        f.in[q] = (const T*)in + (size_t)q * p.geo.N;
        f.out[q] = (T*)out + (size_t)q * p.geo.N;
    }
    for (int a = 0; a < 3; ++a) f.g[a] = p.gfield ? p.gfield + (size_t)a * p.geo.N : nullptr;
    return f;
}

// Planes per block: every block costs about (tz + 2) plane-steps and the
// blocks run in rounds of one per CU, so pick the tz in [16, 64] that
// minimises rounds * (tz + 2) (fewer halo planes vs. a ragged last round).
inline int choose_tz(int columns, int nz, int cus) {
    int best = 32;
    long long best_cost = -1;
    for (int tz = 16; tz <= 64; ++tz) {
        const long long blocks = (long long)columns * ((nz + tz - 1) / tz);
        const long long rounds = (blocks + cus - 1) / cus;
        const long long cost = rounds * (tz + 2);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = tz;
        }
    }
    return best;
}

inline int compute_units() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

template <class S, bool WALLS, bool FIELD>
hipError_t launch_t(const void* in, void* out, const StepParams& p, hipStream_t s) {
    const int tiles_x = (p.geo.n[0] + TX - 1) / TX;
    const int tiles_y = (p.geo.n[1] + TY - 1) / TY;
    const int TZ = choose_tz(tiles_x * tiles_y, p.geo.n[2], compute_units());
    const int tiles_z = (p.geo.n[2] + TZ - 1) / TZ;
    const unsigned nblk = (unsigned)tiles_x * tiles_y * tiles_z;
    if (p.geo.N >= (1LL << 30)) return hipErrorInvalidValue;  // 32-bit node offsets
    const FieldPtrs<typename S::T> f = field_ptrs<S>(in, out, p);
    hipLaunchKernelGGL((update_tiled_kernel<S, WALLS, FIELD>), dim3(nblk), dim3(NTHREADS), 0, s, f, p, tiles_x,
                       tiles_y, tiles_z, TZ);
    return hipGetLastError();
}

template <class S>
hipError_t launch_s(const void* in, void* out, const StepParams& p, hipStream_t s) {
    const bool walls = (p.geo.lo_solid | p.geo.hi_solid) != 0;
    const bool field = p.gfield != nullptr;
    if (walls) return field ? launch_t<S, true, true>(in, out, p, s) : launch_t<S, true, false>(in, out, p, s);
    return field ? launch_t<S, false, true>(in, out, p, s) : launch_t<S, false, false>(in, out, p, s);
}

}  // namespace

template <class S>
hipError_t fixup_s(const void* in, void* out, const StepParams& p, hipStream_t s) {
    if (p.wall_nodes == 0) return hipSuccess;
    const FieldPtrs<typename S::T> f = field_ptrs<S>(in, out, p);
    const int block = 256;
    const unsigned grid = (unsigned)((p.wall_nodes + block - 1) / block);
    hipLaunchKernelGGL(wall_fixup_kernel<S>, dim3(grid), dim3(block), 0, s, f, p, p.wall_nodes);
    return hipGetLastError();
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
