// Tile machinery shared by the tiled update and the tiled adjoint on gfx950:
// tile shape and thread roles, the population polynomial of one node (its
// 17 monomial coefficients and their separable evaluation on the 27
// velocities), slice reductions, addressing helpers and the choice of the
// marched z-extent.
#pragma once
#include <algorithm>
#include <vector>

#include "tslb_internal.h"

namespace tslb {
namespace tile {

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
// 1 (default): the tiled update adds the bounced-back populations of
// wall-adjacent nodes itself, from the populations the node has just built;
// 0: it leaves their raw sums in a side buffer for the wall fix-up launch
#ifndef TSLB_FUSED_WALLS
#define TSLB_FUSED_WALLS 1
#endif
constexpr int TX = TSLB_TILE_X;              // interior tile width (64: one wave per row)
constexpr int TY = TSLB_TILE_Y;              // interior rows
constexpr int LX = TX + 2, LY = TY + 2;      // LDS tile with halo
constexpr int NINT = TX * TY;                // interior threads (whole waves)
constexpr int NHALO = 2 * LX + 2 * TY;       // halo columns
constexpr int NTHREADS = NINT + ((NHALO + 63) / 64) * 64;
static_assert(NINT % 64 == 0, "interior threads must fill whole wavefronts");
static_assert(NTHREADS <= 1024, "a block holds at most 1024 threads");
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
// ORDER 2 keeps the terms up to H2 only (Eq. (fullstrcoll)): the cubic
// monomials vanish and the linear ones reduce to 3 rho (u + g).
// LAT 19 (D3Q19) keeps the third-order content that lattice supports: with
// a3 = rho u u u + sym((1 - omega) Pi u), each pair (a_xxy, a_yzz),
// (a_xzz, a_xyy), (a_yyz, a_xxz) enters as h+ A+ / (2 cs6) + h- A- / (6 cs6)
// (A+- = sum / difference of the pair, h+- the matching Hermite
// combinations, whose norms on D3Q19 are 2 cs6 and 6 cs6), and there is no
// c_x c_y c_z term.  Expanded in monomials: the pair (xxy, yzz) gives
// c_x^2 c_y (27/2 A+ + 9/2 A-), c_y c_z^2 (27/2 A+ - 9/2 A-) and -9 A+ c_y.
template <int ORDER = 3, int LAT = 27>
__host__ __device__ inline void coefficients(const float m[10], const float g[3], float omo, float A[NK]) {
    if constexpr (ORDER == 3 && LAT == 27) {
        // The expansion arranged for few instructions: q_aa = 4.5 (1 - omega)
        // Pi_aa and q_ab = 9 (1 - omega) Pi_ab carry the constants of the
        // quadratic coefficients, v = 4.5 rho u, and the cubic and linear
        // coefficients reuse the quadratic ones:
        //   A_aa  = 4.5 (rho u_a^2 + P_aa) = v_a u_a + q_aa
        //   A_ab  = 9 (rho u_a u_b + P_ab) = 2 v_a u_b + q_ab
        //   A_aab = 27/2 (rho u_a^2 u_b + P_aa u_b + 2 P_ab u_a) = A_aa 3u_b + q_ab 3u_a
        //   A_xyz = 27 (rho u_x u_y u_z + P_xy u_z + P_xz u_y + P_yz u_x)
        //         = A_xy 3u_z + q_xz 3u_y + q_yz 3u_x
        //   A_a   = rho u_a (3 - 9/2 u^2) + u_a (27/2 P_aa - 9/2 tr P) - 9 (P u)_a + 3 rho g_a
        //         = u_a (3 rho - v.u - 4.5 tr P + A_aa) - (q_ab u_b + q_ac u_c) + 3 rho g_a
        //   A_0   = drho - 3/2 (rho u^2 + tr P)
        // with P = (1 - omega) Pi.
        const float dr = m[0], rho = 1.0f + dr;
        const float ux = m[1], uy = m[2], uz = m[3];
        const float o45 = 4.5f * omo, o9 = 9.0f * omo;
        const float qxx = o45 * m[4], qyy = o45 * m[5], qzz = o45 * m[6];
        const float qxy = o9 * m[7], qxz = o9 * m[8], qyz = o9 * m[9];
        const float r45 = 4.5f * rho;
        const float vx = r45 * ux, vy = r45 * uy, vz = r45 * uz;
        const float vu = fmaf(vx, ux, fmaf(vy, uy, vz * uz));  // 4.5 rho u^2
        const float t45 = qxx + qyy + qzz;                      // 4.5 tr P
        A[K000] = fmaf(-1.0f / 3.0f, vu + t45, dr);
        A[K200] = fmaf(vx, ux, qxx);
        A[K020] = fmaf(vy, uy, qyy);
        A[K002] = fmaf(vz, uz, qzz);
        const float wx = vx + vx, wy = vy + vy;
        A[K110] = fmaf(wx, uy, qxy);
        A[K101] = fmaf(wx, uz, qxz);
        A[K011] = fmaf(wy, uz, qyz);
        const float r3 = 3.0f * rho;
        const float base = r3 - vu - t45;
        A[K100] = fmaf(ux, base + A[K200], fmaf(r3, g[0], -fmaf(qxy, uy, qxz * uz)));
        A[K010] = fmaf(uy, base + A[K020], fmaf(r3, g[1], -fmaf(qxy, ux, qyz * uz)));
        A[K001] = fmaf(uz, base + A[K002], fmaf(r3, g[2], -fmaf(qxz, ux, qyz * uy)));
        const float sx = 3.0f * ux, sy = 3.0f * uy, sz = 3.0f * uz;
        A[K210] = fmaf(A[K200], sy, qxy * sx);
        A[K201] = fmaf(A[K200], sz, qxz * sx);
        A[K120] = fmaf(A[K020], sx, qxy * sy);
        A[K021] = fmaf(A[K020], sz, qyz * sy);
        A[K102] = fmaf(A[K002], sx, qxz * sz);
        A[K012] = fmaf(A[K002], sy, qyz * sz);
        A[K111] = fmaf(A[K110], sz, fmaf(qxz, sy, qyz * sx));
        return;
    }

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
    if constexpr (ORDER < 3) {
        A[K100] = 3.0f * (rx + rho * g[0]);
        A[K010] = 3.0f * (ry + rho * g[1]);
        A[K001] = 3.0f * (rz + rho * g[2]);
        A[K210] = A[K201] = A[K120] = A[K021] = A[K102] = A[K012] = A[K111] = 0.0f;
        return;
    }
    if constexpr (LAT == 19) {
        const float axxy = rx * ux * uy + pxx * uy + 2.0f * pxy * ux;
        const float ayzz = ry * uz * uz + pzz * uy + 2.0f * pyz * uz;
        const float axzz = rx * uz * uz + pzz * ux + 2.0f * pxz * uz;
        const float axyy = rx * uy * uy + pyy * ux + 2.0f * pxy * uy;
        const float ayyz = ry * uy * uz + pyy * uz + 2.0f * pyz * uy;
        const float axxz = rx * ux * uz + pxx * uz + 2.0f * pxz * ux;
        const float ap = axxy + ayzz, am = axxy - ayzz;
        const float bp = axzz + axyy, bm = axzz - axyy;
        const float cp = ayyz + axxz, cm = ayyz - axxz;
        A[K210] = 13.5f * ap + 4.5f * am;
        A[K012] = 13.5f * ap - 4.5f * am;
        A[K102] = 13.5f * bp + 4.5f * bm;
        A[K120] = 13.5f * bp - 4.5f * bm;
        A[K021] = 13.5f * cp + 4.5f * cm;
        A[K201] = 13.5f * cp - 4.5f * cm;
        A[K111] = 0.0f;
        A[K100] = 3.0f * (rx + rho * g[0]) - 9.0f * bp;
        A[K010] = 3.0f * (ry + rho * g[1]) - 9.0f * ap;
        A[K001] = 3.0f * (rz + rho * g[2]) - 9.0f * cp;
        return;
    }
}

// Exact scaled weight of a velocity with n0 zero components: 216 w = 4^n0
// on D3Q27; 36 w = 0, 1, 2, 12 on D3Q19 (corners carry no population).
template <int LAT>
__host__ __device__ constexpr float scaled_weight(int n0) {
    if constexpr (LAT == 19) return n0 == 3 ? 12.0f : (n0 == 2 ? 2.0f : (n0 == 1 ? 1.0f : 0.0f));
    return (float)(1 << (2 * n0));
}

// Values of the 2D polynomial Q(cx, cy) = sum b_ab cx^a cy^b on the 3 x 3
// velocity grid of one cz slice, written to G[base + 3 (cy + 1) + (cx + 1)]
// with the exact scaled weight applied (WEIGHTED), or without it for a
// gather that applies the weights itself (add_slice with WEIGHTS).
template <int CZ, int LAT = 27, bool WEIGHTED = true>
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
            const float w = WEIGHTED ? scaled_weight<LAT>((ix == 1) + (iy == 1) + (CZ == 0)) : 1.0f;
            G[I] = (w == 0.0f) ? 0.0f : ((w == 1.0f) ? q[iy] : w * q[iy]);
        }
    }
}

template <int LAT = 27, bool WEIGHTED = true>
__device__ __forceinline__ void populations(const float A[NK], float G[27]) {
    eval_slice<0, LAT, WEIGHTED>(A[K000], A[K100], A[K010], A[K200], A[K020], A[K110], A[K210], A[K120], G);
    const float e00 = A[K000] + A[K002], e10 = A[K100] + A[K102], e01 = A[K010] + A[K012];
    eval_slice<1, LAT, WEIGHTED>(e00 + A[K001], e10 + A[K101], e01 + A[K011], A[K200] + A[K201],
                                 A[K020] + A[K021], A[K110] + A[K111], A[K210], A[K120], G);
    eval_slice<-1, LAT, WEIGHTED>(e00 - A[K001], e10 - A[K101], e01 - A[K011], A[K200] - A[K201],
                                  A[K020] - A[K021], A[K110] - A[K111], A[K210], A[K120], G);
}

// Moments of one arriving cz slice F[cy+1][cx+1], added to the output plane
// accumulator: sum F, sum F c and sum F c c with c = (cx, cy, CZ).  With
// WEIGHTS the values arrive without their lattice weight and the D3Q27
// weights 216 w = 4^(zero components) are applied here, as the separable
// factor 4 of every zero component: each one becomes the constant operand
// of a fused multiply-add that the sum needs anyway, so the weights cost
// no instruction (and, being powers of two, change no rounding).
template <int CZ, bool ASSIGN = false, bool WEIGHTS = false>
__device__ __forceinline__ void add_slice(const float F[3][3], MomentSums& a) {
    constexpr float w0 = WEIGHTS ? 4.0f : 1.0f;           // factor of a zero component
    constexpr float wz = (WEIGHTS && CZ == 0) ? 4.0f : 1.0f;  // of this slice
    float s[3], d[3], t[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        s[r] = F[r][0] + F[r][2];
        d[r] = F[r][2] - F[r][0];
        t[r] = fmaf(w0, F[r][1], s[r]);
    }
    const float m02 = t[2] + t[0];
    const float m00 = fmaf(w0, t[1], m02);
    const float m01 = t[2] - t[0];
    const float m10 = fmaf(w0, d[1], d[0] + d[2]);
    const float m11 = d[2] - d[0];
    const float m20 = fmaf(w0, s[1], s[0] + s[2]);
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
        a.d = fmaf(wz, m00, a.d);
        a.j[0] = fmaf(wz, m10, a.j[0]);
        a.j[1] = fmaf(wz, m01, a.j[1]);
        a.s[0] = fmaf(wz, m20, a.s[0]);
        a.s[1] = fmaf(wz, m02, a.s[1]);
        a.s[3] = fmaf(wz, m11, a.s[3]);
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
// That pays when a grid row is a whole number of 128-B cache lines; with
// other row lengths a wave's row straddles lines that the neighbouring tile
// completes, and plain stores let L2 merge the two halves before they go to
// memory (the launch decides, NT).
template <bool NT, class T>
__device__ __forceinline__ void store_out(T* p, T v) {
    if constexpr (NT && TSLB_NT_STORE) {
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

// The stored values of node n, left unconverted: a caller that loads the
// next plane ahead keeps them in flight until the plane's build converts
// them (a conversion right after the loads would wait for them there).
template <class S>
__device__ __forceinline__ void load_raw(const FieldPtrs<typename S::T>& f, unsigned n, typename S::T r[10]) {
    unsigned off = n * (unsigned)sizeof(typename S::T);
    // keep the offset opaque so that each load is one scalar base plus this
    // shared offset (no per-field 64-bit addresses carried across planes)
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int q = 0; q < 10; ++q) r[q] = ld_at(f.in[q], off);
}

// Converted values of load_raw.  drho and u get their scales; Pi^neq is
// left unscaled: the caller folds 1 / scale[2] into 1 - omega, the only
// factor Pi^neq meets in coefficients() (exact, a power of two).
template <class S>
__device__ __forceinline__ void convert_raw(const typename S::T r[10], const StepParams& p, float m[10]) {
    m[0] = S::load(r[0], p.inv_scale[0]);
#pragma unroll
    for (int q = 1; q < 4; ++q) m[q] = S::load(r[q], p.inv_scale[1]);
#pragma unroll
    for (int q = 4; q < 10; ++q) m[q] = S::convert(r[q]);
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

// Blocks of the tiled kernels that one CU holds at once: bounded by LDS
// (160 KB per CU) and by the waves the register budget allows (4 SIMDs x
// TSLB_WAVES_PER_EU waves).
constexpr int kLdsBytes = NSLOT * LY * LX * 4;
constexpr int kBlocksPerCu = (163840 / kLdsBytes) < ((4 * TSLB_WAVES_PER_EU) / (NTHREADS / 64))
                                 ? (163840 / kLdsBytes)
                                 : ((4 * TSLB_WAVES_PER_EU) / (NTHREADS / 64));
static_assert(kBlocksPerCu >= 1, "a tile must fit one CU");

// Work list of the tiled update.  Every block of the grid marches a short
// list of column segments (tile column, first plane, end plane); a segment
// of L planes costs about L + 2 plane-steps (one halo plane at each end).
// Tiles of tz planes are dealt in whole rounds, one tile per block and
// round; round r gives XCD k a contiguous run of tiles, so the blocks of one
// XCD march neighbouring columns in step and read each other's halo columns
// from its L2.  The tiles left over after the last whole round are cut into
// `split` parts along z, and the parts, part index major, are dealt in
// rounds the same way: without that cut a grid whose tile count is not a
// multiple of the resident blocks leaves most CUs idle in its last round.
// The (tz, split) with the smallest largest block cost is taken.  Entry
// b * nseg + k is segment k of block b ({column, z begin, z end, 0}; column
// -1 ends a shorter list); block ids are dealt round-robin to the 8 XCDs.
struct Schedule {
    std::vector<int4> seg;
    int grid = 0, nseg = 0, tz = 0, split = 1;
    long long cost = 0;
};

// The schedule for one (tz, split); with build == false only its cost (the
// largest per-block sum of L + 2 over the block's segments) and shape.
inline Schedule schedule_for(int columns, int nz, int resident, int tz, int split, bool build) {
    const int tiles_z = (nz + tz - 1) / tz;
    const long long ntiles = (long long)columns * tiles_z;
    const int nb = resident;  // a multiple of 8
    const long long rounds = ntiles / nb;
    std::vector<long long> cost(nb, 0);
    std::vector<int> count(nb, 0);
    std::vector<std::vector<int4>> lists(build ? nb : 0);
    // item i of a round of n items: XCD i / per, slot i % per, per = n / 8
    // rounded up, so every XCD takes a contiguous run of the round's items
    auto deal = [&](long long i, long long n, int col, int z0, int z1) {
        const long long per = (n + 7) / 8;
        const long long b = 8 * (i % per) + i / per;
        cost[b] += z1 - z0 + 2;
        count[b] += 1;
        if (build) lists[b].push_back(make_int4(col, z0, z1, 0));
    };
    auto tile = [&](long long t, int& col, int& z0, int& z1) {
        col = (int)(t % columns);
        z0 = (int)(t / columns) * tz;
        z1 = std::min(z0 + tz, nz);
    };
    for (long long t = 0; t < rounds * nb; ++t) {
        int col, z0, z1;
        tile(t, col, z0, z1);
        deal(t % nb, nb, col, z0, z1);
    }
    // leftover tiles, each cut into `split` parts along z (part index major)
    const long long left = ntiles - rounds * nb;
    const long long parts = left * split;
    for (long long q = 0; q < parts; ++q) {
        const long long t = rounds * nb + q % left;
        const int k = (int)(q / left);
        int col, z0, z1;
        tile(t, col, z0, z1);
        const int len = z1 - z0;
        const int a = z0 + (int)((long long)len * k / split), e = z0 + (int)((long long)len * (k + 1) / split);
        if (a == e) continue;  // a part of a short tile may be empty
        const long long r0 = q / nb * nb;
        deal(q - r0, std::min<long long>(nb, parts - r0), col, a, e);
    }
    Schedule s;
    s.tz = tz;
    s.split = split;
    int last = -1;
    for (int b = 0; b < nb; ++b) {
        s.cost = std::max(s.cost, cost[b]);
        s.nseg = std::max(s.nseg, count[b]);
        if (count[b] > 0) last = b;
    }
    s.grid = (last + 8) & ~7;
    if (build) {
        s.seg.assign((size_t)s.grid * s.nseg, make_int4(-1, 0, 0, 0));
        for (int b = 0; b < s.grid; ++b)
            for (size_t k = 0; k < lists[b].size(); ++k) s.seg[(size_t)b * s.nseg + k] = lists[b][k];
    }
    return s;
}

inline Schedule build_schedule(int columns, int nz, int resident) {
    int best_tz = 1, best_split = 1;
    long long best_cost = -1;
    int best_nseg = 0;
    for (int tz = 1; tz <= 64 && tz <= nz; ++tz) {
        const long long left = ((long long)columns * ((nz + tz - 1) / tz)) % resident;
        for (int split = 1; split <= (left ? std::min(tz, 8) : 1); ++split) {
            const Schedule s = schedule_for(columns, nz, resident, tz, split, false);
            if (best_cost < 0 || s.cost < best_cost || (s.cost == best_cost && s.nseg < best_nseg)) {
                best_cost = s.cost;
                best_nseg = s.nseg;
                best_tz = tz;
                best_split = split;
            }
        }
    }
    return schedule_for(columns, nz, resident, best_tz, best_split, true);
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

// Reverse-mode derivative of coefficients(): given L[k] = dF/dA_k, the
// sensitivities of F to the node's stored moments (drho, u, Pi) and to its
// acceleration g.  Written out term by term from coefficients() (the
// products are differentiated in the order they are formed there).
__host__ __device__ inline void coefficients_vjp(const float L[NK], const float m[10], const float g[3], float omo,
                                                 float lam[10], float lg[3]) {
    const float r = 1.0f + m[0];
    const float ux = m[1], uy = m[2], uz = m[3];
    const float pxx = omo * m[4], pyy = omo * m[5], pzz = omo * m[6];
    const float pxy = omo * m[7], pxz = omo * m[8], pyz = omo * m[9];
    const float uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
    const float u2 = uxx + uyy + uzz;
    const float tr = pxx + pyy + pzz;
    const float base = 3.0f - 4.5f * u2;
    float gr = 0, gux = 0, guy = 0, guz = 0, gu2 = 0, gtr = 0, gbase = 0;
    float gpxx = 0, gpyy = 0, gpzz = 0, gpxy = 0, gpxz = 0, gpyz = 0;
    float gdr = L[K000];
    // A000 = drho - 1.5 (r u2 + tr)
    gr += -1.5f * u2 * L[K000];
    gu2 += -1.5f * r * L[K000];
    gtr += -1.5f * L[K000];
    // A_aa = 4.5 (r u_a^2 + P_aa)
    gr += 4.5f * (uxx * L[K200] + uyy * L[K020] + uzz * L[K002]);
    gux += 9.0f * r * ux * L[K200];
    guy += 9.0f * r * uy * L[K020];
    guz += 9.0f * r * uz * L[K002];
    gpxx += 4.5f * L[K200];
    gpyy += 4.5f * L[K020];
    gpzz += 4.5f * L[K002];
    // A_ab = 9 (r u_a u_b + P_ab)
    gr += 9.0f * (ux * uy * L[K110] + ux * uz * L[K101] + uy * uz * L[K011]);
    gux += 9.0f * r * (uy * L[K110] + uz * L[K101]);
    guy += 9.0f * r * (ux * L[K110] + uz * L[K011]);
    guz += 9.0f * r * (ux * L[K101] + uy * L[K011]);
    gpxy += 9.0f * L[K110];
    gpxz += 9.0f * L[K101];
    gpyz += 9.0f * L[K011];
    // A_a = r u_a (base + 4.5 u_a^2) + u_a (13.5 P_aa - 4.5 tr) - 9 (P u)_a + 3 r g_a
    const float la[3] = {L[K100], L[K010], L[K001]};
    const float u[3] = {ux, uy, uz};
    const float paa[3] = {pxx, pyy, pzz};
    float gu[3] = {0, 0, 0}, gpaa[3] = {0, 0, 0}, gpu[3];
    for (int a = 0; a < 3; ++a) {
        const float e = base + 4.5f * u[a] * u[a];
        gr += (u[a] * e + 3.0f * g[a]) * la[a];
        gu[a] += (r * e + 9.0f * r * u[a] * u[a] + 13.5f * paa[a] - 4.5f * tr) * la[a];
        gbase += r * u[a] * la[a];
        gpaa[a] += 13.5f * u[a] * la[a];
        gtr += -4.5f * u[a] * la[a];
        gpu[a] = -9.0f * la[a];
        lg[a] = 3.0f * r * la[a];
    }
    gux += gu[0];
    guy += gu[1];
    guz += gu[2];
    gpxx += gpaa[0];
    gpyy += gpaa[1];
    gpzz += gpaa[2];
    gu2 += -4.5f * gbase;
    // (P u)_x = pxx ux + pxy uy + pxz uz, and its y, z rows
    gpxx += ux * gpu[0];
    gpxy += uy * gpu[0] + ux * gpu[1];
    gpxz += uz * gpu[0] + ux * gpu[2];
    gpyy += uy * gpu[1];
    gpyz += uz * gpu[1] + uy * gpu[2];
    gpzz += uz * gpu[2];
    gux += pxx * gpu[0] + pxy * gpu[1] + pxz * gpu[2];
    guy += pxy * gpu[0] + pyy * gpu[1] + pyz * gpu[2];
    guz += pxz * gpu[0] + pyz * gpu[1] + pzz * gpu[2];
    // A_aab = 13.5 (r u_a^2 u_b + P_aa u_b + 2 P_ab u_a)
    {
        const float l = 13.5f * L[K210];  // cx^2 cy
        gr += uxx * uy * l;
        gux += (2.0f * r * ux * uy + 2.0f * pxy) * l;
        guy += (r * uxx + pxx) * l;
        gpxx += uy * l;
        gpxy += 2.0f * ux * l;
    }
    {
        const float l = 13.5f * L[K201];  // cx^2 cz
        gr += uxx * uz * l;
        gux += (2.0f * r * ux * uz + 2.0f * pxz) * l;
        guz += (r * uxx + pxx) * l;
        gpxx += uz * l;
        gpxz += 2.0f * ux * l;
    }
    {
        const float l = 13.5f * L[K120];  // cy^2 cx
        gr += uyy * ux * l;
        guy += (2.0f * r * uy * ux + 2.0f * pxy) * l;
        gux += (r * uyy + pyy) * l;
        gpyy += ux * l;
        gpxy += 2.0f * uy * l;
    }
    {
        const float l = 13.5f * L[K021];  // cy^2 cz
        gr += uyy * uz * l;
        guy += (2.0f * r * uy * uz + 2.0f * pyz) * l;
        guz += (r * uyy + pyy) * l;
        gpyy += uz * l;
        gpyz += 2.0f * uy * l;
    }
    {
        const float l = 13.5f * L[K102];  // cz^2 cx
        gr += uzz * ux * l;
        guz += (2.0f * r * uz * ux + 2.0f * pxz) * l;
        gux += (r * uzz + pzz) * l;
        gpzz += ux * l;
        gpxz += 2.0f * uz * l;
    }
    {
        const float l = 13.5f * L[K012];  // cz^2 cy
        gr += uzz * uy * l;
        guz += (2.0f * r * uz * uy + 2.0f * pyz) * l;
        guy += (r * uzz + pzz) * l;
        gpzz += uy * l;
        gpyz += 2.0f * uz * l;
    }
    {
        const float l = 27.0f * L[K111];  // cx cy cz
        gr += ux * uy * uz * l;
        gux += (r * uy * uz + pyz) * l;
        guy += (r * ux * uz + pxz) * l;
        guz += (r * ux * uy + pxy) * l;
        gpxy += uz * l;
        gpxz += uy * l;
        gpyz += ux * l;
    }
    // u2 = |u|^2, tr = trace, r = 1 + drho, P = (1 - omega) Pi
    gux += 2.0f * ux * gu2;
    guy += 2.0f * uy * gu2;
    guz += 2.0f * uz * gu2;
    gpxx += gtr;
    gpyy += gtr;
    gpzz += gtr;
    lam[0] = gdr + gr;
    lam[1] = gux;
    lam[2] = guy;
    lam[3] = guz;
    lam[4] = omo * gpxx;
    lam[5] = omo * gpyy;
    lam[6] = omo * gpzz;
    lam[7] = omo * gpxy;
    lam[8] = omo * gpxz;
    lam[9] = omo * gpyz;
}

}  // namespace tile
}  // namespace tslb
