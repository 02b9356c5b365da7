// D2Q9 form of the moment-only thread-safe update (the two-dimensional
// counterpart of D3Q27 that Section 2.2 names): the tensor product of the
// three-point weights in x and y, the same Hermite reconstruction (up to
// third order; H_xxx vanishes on this lattice as on D3Q27) and the same
// BGK relaxation and forcing.  The state keeps the 10-field layout with
// nz = 1; the update reads and writes the six fields drho, u_x, u_y,
// Pi_xx, Pi_yy, Pi_xy only (u_z and the Pi components with a z index stay
// zero).
//
// Kernel shape: one wavefront owns a strip of 64 x-columns (whole cache
// lines) and marches a segment of rows along y.  For every row it builds
// the 9 populations of its 64 nodes (scaled deviations G = 36 w P,
// 36 w = 4^n0 exact), moves the ones with c_x != 0 to their x-neighbour with
// a cross-lane permute (no LDS allocation, no block barrier; the two edge
// lanes rebuild the three values that enter from the neighbouring strips),
// and adds each c_y slice into the rolling accumulator of the row it arrives
// in (rows y - 1, y, y + 1).  Row y - 1 is then complete and is
// finalised and stored.  Walls: wall nodes are stored as the rest state and
// emit nothing; a fluid node next to a wall adds its own bounced-back
// populations, straight from the nine it has just built, to its own row
// (half-way bounce-back).
#include "tslb_internal.h"

namespace tslb {
namespace {

#ifndef TSLB_D2_WAVES
#define TSLB_D2_WAVES 32
#endif
constexpr int kD2Block = 256;          // four independent wavefronts
constexpr int kStrip = 64;             // columns per wavefront: one per lane, whole cache lines


// Moment sums of the arriving scaled deviations (2D).
struct Sums2 {
    float d, jx, jy, sxx, syy, sxy;
    __device__ __forceinline__ void zero() { d = jx = jy = sxx = syy = sxy = 0.0f; }
    template <int CX, int CY>
    __device__ __forceinline__ void add(float f) {
        d += f;
        if (CX) {
            jx += CX * f;
            sxx += f;
        }
        if (CY) {
            jy += CY * f;
            syy += f;
        }
        if (CX * CY) sxy += CX * CY * f;
    }
};

// Population polynomial of one node, G(c) = 36 w(c) P(c): P is the
// polynomial of the D3Q27 kernels with every z component zero (the
// expression does not depend on the dimension),
//   P = b00 + b10 cx + b01 cy + b20 cx^2 + b02 cy^2 + b11 cx cy
//       + b21 cx^2 cy + b12 cx cy^2,
// from the equilibrium rho [3 cu + 9/2 cu^2 - 3/2 u^2 + 9/2 cu^3 - 9/2 cu u^2]
// and the non-equilibrium part (1 - omega) [9/2 cPc - 3/2 tr Pi +
// 27/2 cPc cu - 9/2 tr Pi cu - 9 c.Pi u] with c_a^3 = c_a, plus 3 rho c.g.
// ORDER 2 keeps the terms up to H2 (the cubic monomials vanish and the
// linear ones reduce to 3 rho (u + g)).  m = (drho, u_x, u_y, Pi_xx, Pi_yy,
// Pi_xy); b = (b00, b10, b01, b20, b02, b11, b21, b12).
template <int ORDER>
__device__ __forceinline__ void coefficients2(const float m[6], float gx, float gy, float omo, float b[8]) {
    const float dr = m[0], rho = 1.0f + dr, ux = m[1], uy = m[2];
    const float pxx = omo * m[3], pyy = omo * m[4], pxy = omo * m[5];
    const float rx = rho * ux, ry = rho * uy;
    const float u2 = ux * ux + uy * uy, tr = pxx + pyy;
    b[0] = dr - 1.5f * (rho * u2 + tr);
    b[3] = 4.5f * (rx * ux + pxx);
    b[4] = 4.5f * (ry * uy + pyy);
    b[5] = 9.0f * (rx * uy + pxy);
    if constexpr (ORDER < 3) {
        b[1] = 3.0f * (rx + rho * gx);
        b[2] = 3.0f * (ry + rho * gy);
        b[6] = b[7] = 0.0f;
        return;
    }
    // 27/2 (rho u_a^2 u_b + Pi_aa u_b + 2 Pi_ab u_a) = 3 b_aa u_b + 27 Pi_ab u_a;
    // the Pi_aa u_a terms of the linear coefficients collapse into b_aa u_a
    const float base = 3.0f - 4.5f * u2, t45 = 4.5f * tr, qxy = 27.0f * pxy;
    b[1] = rx * base + ux * (b[3] - t45) - 9.0f * pxy * uy + 3.0f * rho * gx;
    b[2] = ry * base + uy * (b[4] - t45) - 9.0f * pxy * ux + 3.0f * rho * gy;
    b[6] = 3.0f * b[3] * uy + qxy * ux;
    b[7] = 3.0f * b[4] * ux + qxy * uy;
}

// G[3 (cy + 1) + (cx + 1)] = 4^n0 P(cx, cy) (36 w = 4^n0, n0 the number of
// zero components): along x for each power of cy, then along y.
__device__ __forceinline__ void populations2(const float b[8], float G[9]) {
    const float s0 = b[0] + b[3], s1 = b[2] + b[6];
    const float r0[3] = {s0 - b[1], b[0], s0 + b[1]};
    const float r1[3] = {s1 - b[5], b[2], s1 + b[5]};
    const float r2[3] = {b[4] - b[7], b[4], b[4] + b[7]};
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) {
        const float t = r0[ix] + r2[ix];
        const float q[3] = {t - r1[ix], r0[ix], t + r1[ix]};
#pragma unroll
        for (int iy = 0; iy < 3; ++iy) {
            const int n0 = (ix == 1) + (iy == 1);
            G[3 * iy + ix] = n0 == 0 ? q[iy] : (float)(1 << (2 * n0)) * q[iy];
        }
    }
}

__device__ __forceinline__ float from_lane(int src_lane, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

// Per-field base pointers of the six stored D2Q9 fields (drho, u_x, u_y,
// Pi_xx, Pi_yy, Pi_xy: fields 0, 1, 2, 4, 5, 7 of the ten-field state) and
// of the force field, passed as a kernel argument so every base sits in
// scalar registers and each access is that base plus one 32-bit byte offset.
template <class T>
struct Fields2 {
    const T* in[6];
    T* out[6];
    const float* g[2];
};

template <class S>
__device__ __forceinline__ void load6(const Fields2<typename S::T>& f, unsigned off, const StepParams& p, float m[6]) {
    using T = typename S::T;
    m[0] = S::load(*(const T*)((const char*)f.in[0] + off), p.inv_scale[0]);
#pragma unroll
    for (int k = 1; k < 3; ++k) m[k] = S::load(*(const T*)((const char*)f.in[k] + off), p.inv_scale[1]);
#pragma unroll
    for (int k = 3; k < 6; ++k) m[k] = S::load(*(const T*)((const char*)f.in[k] + off), p.inv_scale[2]);
}

__device__ __forceinline__ int wrap_clamp(int v, int n, bool periodic) {
    if (periodic) {
        v %= n;
        return v < 0 ? v + n : v;
    }
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// Output stores, non-temporal (the new level is not read again by this
// launch) when every grid row is a whole number of 128-B cache lines, plain
// otherwise (a strip's row then straddles lines its neighbour completes).
template <bool NT, class T>
__device__ __forceinline__ void out_store(T* p, T v) {
    if constexpr (!NT)
        *p = v;
    else if constexpr (sizeof(T) == 4)
        __builtin_nontemporal_store(__builtin_bit_cast(float, v), reinterpret_cast<float*>(p));
    else
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), reinterpret_cast<unsigned short*>(p));
}

template <class S, int ORDER, bool FIELD, bool NT>
__global__ void __launch_bounds__(kD2Block) update_d2q9_kernel(const Fields2<typename S::T> f, StepParams p, int strips,
                                                               int segments, int seg_rows) {
    using T = typename S::T;
    const Geometry& g = p.geo;
    const int nx = g.n[0], ny = g.n[1];
    const int lane = threadIdx.x & 63;
    // Block ids are dealt round-robin to the 8 XCDs (the grid is a multiple
    // of 8 blocks); each XCD takes a contiguous run of blocks, so the strips
    // that march side by side share an L2 and the halo columns the edge
    // lanes read are mostly hits.
    const int per = (int)(gridDim.x >> 3);
    const int vb = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    const int item = vb * (kD2Block / 64) + (int)(threadIdx.x >> 6);
    if (item >= strips * segments) return;  // whole wavefronts leave together
    const int strip = item % strips, seg = item / strips;
    const int y0 = seg * seg_rows, y1 = min(y0 + seg_rows, ny);
    const int x0 = strip * kStrip, gx = x0 + lane;
    const bool px = (g.periodic & 1) != 0, py = (g.periodic & 2) != 0;
    // lanes past the last column build the node the periodic wrap or the
    // clamp puts there (its populations still reach the last column)
    const int x = wrap_clamp(gx, nx, px);
    const bool interior = gx < nx;
    // the edge lanes also rebuild the populations that enter the strip from
    // the neighbouring columns: lane 0 those with c_x = +1 of node x0 - 1,
    // lane 63 those with c_x = -1 of node x0 + 64
    const bool edge = lane == 0 || lane == kStrip - 1;
    const int hx = wrap_clamp(lane == 0 ? x0 - 1 : x0 + kStrip, nx, px);
    const float hs = lane == 0 ? 1.0f : -1.0f;
    const bool hsolid_col = (hx == 0 && (g.lo_solid & 1)) || (hx == nx - 1 && (g.hi_solid & 1));
    const bool col_solid = (x == 0 && (g.lo_solid & 1)) || (x == nx - 1 && (g.hi_solid & 1));
    const bool fluid_col = interior && !col_solid && !(x == 0 && (g.lo_ghost & 1)) && !(x == nx - 1 && (g.hi_ghost & 1));
    const bool wl = (g.lo_solid & 1) && x == 1, wr = (g.hi_solid & 1) && x == nx - 2;
    const float omo = omo_at(p, 0);
    // arrivals at this lane: the population with c_x = +1 comes from the
    // lane on the left (lane 0: its halo value), c_x = -1 from the lane on
    // the right (lane 63: its halo value)
    const int left = (lane + 63) & 63, right = (lane + 1) & 63;
    auto from_left = [&](float v, float h) {
        const float w = from_lane(left, v);
        return lane == 0 ? h : w;
    };
    auto from_right = [&](float v, float h) {
        const float w = from_lane(right, v);
        return lane == kStrip - 1 ? h : w;
    };

    auto row = [&](int yp, Sums2& aprev, Sums2& acur, Sums2& anext) {
        const int y = wrap_clamp(yp, ny, py);
        const unsigned off = (unsigned)(x + nx * y) * (unsigned)sizeof(T);  // < 2^32: N < 2^30
        float m[6];
        load6<S>(f, off, p, m);
        const bool solid = col_solid || (y == 0 && (g.lo_solid & 2)) || (y == ny - 1 && (g.hi_solid & 2));
        float gxv = 0.0f, gyv = 0.0f;
        if (!solid) {
            gxv = FIELD ? *(const float*)((const char*)f.g[0] + (off / sizeof(T)) * 4u) : p.force[0];
            gyv = FIELD ? *(const float*)((const char*)f.g[1] + (off / sizeof(T)) * 4u) : p.force[1];
        }
        float b[8];
        coefficients2<ORDER>(m, gxv, gyv, omo, b);
        float G[9];
        populations2(b, G);
        // halo populations H[cy + 1] = 36 w P(hs, cy) of node (hx, y), with
        // P(s, cy) = r0 + cy r1 + cy^2 r2 and 36 w = 4^(cy == 0)
        float H[3] = {0.0f, 0.0f, 0.0f};
        if (edge) {
            float mh[6], bh[8];
            const unsigned hoff = (unsigned)(hx + nx * y) * (unsigned)sizeof(T);
            load6<S>(f, hoff, p, mh);
            const bool hsolid = hsolid_col || (y == 0 && (g.lo_solid & 2)) || (y == ny - 1 && (g.hi_solid & 2));
            float hgx = 0.0f, hgy = 0.0f;
            if (!hsolid) {
                hgx = FIELD ? *(const float*)((const char*)f.g[0] + (hoff / sizeof(T)) * 4u) : p.force[0];
                hgy = FIELD ? *(const float*)((const char*)f.g[1] + (hoff / sizeof(T)) * 4u) : p.force[1];
            }
            coefficients2<ORDER>(mh, hgx, hgy, omo, bh);
            const float r0 = bh[0] + hs * bh[1] + bh[3], r1 = bh[2] + hs * bh[5] + bh[6], r2 = bh[4] + hs * bh[7];
            const float t2 = r0 + r2;
            H[0] = t2 - r1;
            H[1] = 4.0f * r0;
            H[2] = t2 + r1;
        }
        // slice c_y = -1 (I = 0, 1, 2) arrives in row yp - 1
        aprev.template add<-1, -1>(from_right(G[0], H[0]));
        aprev.template add<0, -1>(G[1]);
        aprev.template add<1, -1>(from_left(G[2], H[0]));
        // slice c_y = 0 (I = 3, 4, 5) stays in row yp
        acur.template add<-1, 0>(from_right(G[3], H[1]));
        acur.template add<0, 0>(G[4]);
        acur.template add<1, 0>(from_left(G[5], H[1]));
        // slice c_y = +1 (I = 6, 7, 8) starts row yp + 1
        anext.zero();
        anext.template add<-1, 1>(from_right(G[6], H[2]));
        anext.template add<0, 1>(G[7]);
        anext.template add<1, 1>(from_left(G[8], H[2]));
        // half-way bounce-back: a fluid node next to a wall receives its own
        // population along -c for every c whose upstream node x - c is a
        // wall; it arrives in the node's own row
        const bool wb = (g.lo_solid & 2) && yp == 1, wt = (g.hi_solid & 2) && yp == ny - 2;
        if (fluid_col && !solid && (wl || wr || wb || wt)) {
#define TSLB_BB(I, X, Y) \
    if ((X == 1 && wl) || (X == -1 && wr) || (Y == 1 && wb) || (Y == -1 && wt)) acur.template add<X, Y>(G[8 - I]);
            TSLB_BB(0, -1, -1)
            TSLB_BB(1, 0, -1)
            TSLB_BB(2, 1, -1)
            TSLB_BB(3, -1, 0)
            TSLB_BB(5, 1, 0)
            TSLB_BB(6, -1, 1)
            TSLB_BB(7, 0, 1)
            TSLB_BB(8, 1, 1)
#undef TSLB_BB
        }

        const int yo = yp - 1;  // row yp - 1 is complete
        if (!(fluid_col && yo >= y0 && yo < y1)) return;
        if ((yo == 0 && ((g.lo_solid | g.lo_ghost) & 2)) || (yo == ny - 1 && ((g.hi_solid | g.hi_ghost) & 2))) return;
        const Sums2& a = aprev;
        // drho' = D/36, u' = J/(36 + D), Pi' = (S - J u' - D/3 delta)/36
        const float den = 36.0f + a.d;
        float inv = __builtin_amdgcn_rcpf(den);
        inv = inv * fmaf(-den, inv, 2.0f);
        const float ux = a.jx * inv, uy = a.jy * inv, d3 = a.d * (1.0f / 3.0f);
        constexpr float k36 = 1.0f / 36.0f;
        const unsigned oo = (unsigned)(x + nx * yo) * (unsigned)sizeof(T);
        out_store<NT>((T*)((char*)f.out[0] + oo), S::store(a.d * k36, p.scale[0]));
        out_store<NT>((T*)((char*)f.out[1] + oo), S::store(ux, p.scale[1]));
        out_store<NT>((T*)((char*)f.out[2] + oo), S::store(uy, p.scale[1]));
        out_store<NT>((T*)((char*)f.out[3] + oo), S::store((a.sxx - a.jx * ux - d3) * k36, p.scale[2]));
        out_store<NT>((T*)((char*)f.out[4] + oo), S::store((a.syy - a.jy * uy - d3) * k36, p.scale[2]));
        out_store<NT>((T*)((char*)f.out[5] + oo), S::store((a.sxy - a.jx * uy) * k36, p.scale[2]));
    };

    Sums2 a0, a1, a2;
    a0.zero();
    a1.zero();
    for (int yp = y0 - 1; yp <= y1; yp += 3) {
        row(yp, a0, a1, a2);
        if (yp + 1 > y1) break;
        row(yp + 1, a1, a2, a0);
        if (yp + 2 > y1) break;
        row(yp + 2, a2, a0, a1);
    }
}

template <class S, int ORDER>
hipError_t launch_o(const void* in, void* out, const StepParams& p, int strips, int segments, int seg_rows,
                    hipStream_t s) {
    using T = typename S::T;
    const int waves = strips * segments;
    const unsigned blocks = (unsigned)((waves + kD2Block / 64 - 1) / (kD2Block / 64));
    const unsigned grid = (blocks + 7u) & ~7u;  // a multiple of 8: whole runs per XCD
    const size_t N = (size_t)p.geo.N;
    Fields2<T> f;
    const int field[6] = {0, 1, 2, 4, 5, 7};
    for (int k = 0; k < 6; ++k) {
        f.in[k] = (const T*)in + field[k] * N;
        f.out[k] = (T*)out + field[k] * N;
    }
    for (int a = 0; a < 2; ++a) f.g[a] = p.gfield ? p.gfield + a * N : nullptr;
    const bool nt = ((long long)p.geo.n[0] * (long long)sizeof(T)) % 128 == 0;
    if (p.gfield && nt)
        hipLaunchKernelGGL((update_d2q9_kernel<S, ORDER, true, true>), dim3(grid), dim3(kD2Block), 0, s, f, p, strips,
                           segments, seg_rows);
    else if (p.gfield)
        hipLaunchKernelGGL((update_d2q9_kernel<S, ORDER, true, false>), dim3(grid), dim3(kD2Block), 0, s, f, p, strips,
                           segments, seg_rows);
    else if (nt)
        hipLaunchKernelGGL((update_d2q9_kernel<S, ORDER, false, true>), dim3(grid), dim3(kD2Block), 0, s, f, p, strips,
                           segments, seg_rows);
    else
        hipLaunchKernelGGL((update_d2q9_kernel<S, ORDER, false, false>), dim3(grid), dim3(kD2Block), 0, s, f, p, strips,
                           segments, seg_rows);
    return hipGetLastError();
}

template <class S>
hipError_t launch_s(const void* in, void* out, const StepParams& p, int strips, int segments, int seg_rows,
                    hipStream_t s) {
    return p.order == 2 ? launch_o<S, 2>(in, out, p, strips, segments, seg_rows, s)
                        : launch_o<S, 3>(in, out, p, strips, segments, seg_rows, s);
}

}  // namespace

hipError_t launch_update_d2q9(int storage, const void* in, void* out, const StepParams& p, hipStream_t s) {
    const int nx = p.geo.n[0], ny = p.geo.n[1];
    if (p.geo.n[2] != 1 || p.geo.N >= (1LL << 30)) return hipErrorInvalidValue;  // 32-bit byte offsets
    const int strips = (nx + kStrip - 1) / kStrip;
    // rows per segment: enough wavefronts to fill the chip (TSLB_D2_WAVES
    // per CU, at most 8 per SIMD at <= 64 VGPRs) while keeping the two halo
    // rows of a segment a small overhead
    const long long target = 256LL * TSLB_D2_WAVES;
    long long segments = (target + strips - 1) / strips;
    int seg_rows = (int)((ny + segments - 1) / segments);
    if (seg_rows < 16) seg_rows = 16;
    segments = (ny + seg_rows - 1) / seg_rows;
    switch (storage) {
    case 0: return launch_s<StoreF32>(in, out, p, strips, (int)segments, seg_rows, s);
    case 1: return launch_s<StoreF16>(in, out, p, strips, (int)segments, seg_rows, s);
    case 2: return launch_s<StoreBF16>(in, out, p, strips, (int)segments, seg_rows, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace tslb
