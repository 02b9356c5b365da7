// D2Q9 form of the moment-only thread-safe update (the two-dimensional
// counterpart of D3Q27 that Section 2.2 names): the tensor product of the
// three-point weights in x and y, the same Hermite reconstruction (up to
// third order; H_xxx vanishes on this lattice as on D3Q27) and the same
// BGK relaxation and forcing.  The state keeps the 10-field layout with
// nz = 1; the update reads and writes the six fields drho, u_x, u_y,
// Pi_xx, Pi_yy, Pi_xy only (u_z and the Pi components with a z index stay
// zero).
//
// Kernel shape: one wavefront owns a strip of 62 interior x-columns plus a
// halo lane on each side and marches a segment of rows along y.  For every
// row it builds the 9 populations of its 64 nodes (scaled deviations
// G = 36 w P, 36 w = 4^n0 exact), moves the ones with c_x != 0 to their
// x-neighbour with a cross-lane permute (no LDS allocation, no block
// barrier), and adds each c_y slice into the rolling accumulator of the row
// it arrives in (rows y - 1, y, y + 1).  Row y - 1 is then complete and is
// finalised and stored.  Walls: wall nodes are stored as the rest state and
// emit nothing; a fluid node next to a wall adds its own bounced-back
// populations at finalisation (half-way bounce-back).
#include "tslb_internal.h"

namespace tslb {
namespace {

constexpr int kD2Block = 256;          // four independent wavefronts
constexpr int kStrip = 62;             // interior columns per wavefront

__device__ __forceinline__ constexpr int cx9(int i) { return i % 3 - 1; }
__device__ __forceinline__ constexpr int cy9(int i) { return i / 3 - 1; }

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

// Population polynomial of one node: P(c) as in the D3Q27 kernels (the
// expression does not depend on the dimension), returned as G = 4^n0 P.
struct Terms2 {
    float dr, rho, ux, uy, u2, pxx, pyy, pxy, trp, pux, puy, rgx, rgy, omo;
};

__device__ __forceinline__ Terms2 terms2(const float m[6], float gx, float gy, float omo) {
    Terms2 t;
    t.dr = m[0];
    t.rho = 1.0f + m[0];
    t.ux = m[1];
    t.uy = m[2];
    t.u2 = m[1] * m[1] + m[2] * m[2];
    t.pxx = m[3];
    t.pyy = m[4];
    t.pxy = m[5];
    t.trp = m[3] + m[4];
    t.pux = m[3] * m[1] + m[5] * m[2];
    t.puy = m[5] * m[1] + m[4] * m[2];
    t.rgx = t.rho * gx;
    t.rgy = t.rho * gy;
    t.omo = omo;
    return t;
}

template <int I, int ORDER>
__device__ __forceinline__ float emit9(const Terms2& t) {
    constexpr int X = cx9(I), Y = cy9(I);
    constexpr float W = (float)(1 << (2 * ((X == 0) + (Y == 0))));
    const float cu = X * t.ux + Y * t.uy;
    const float cpc = X * X * t.pxx + Y * Y * t.pyy + 2.0f * X * Y * t.pxy;
    float eq = cu * (3.0f + 4.5f * cu) - 1.5f * t.u2;
    float neq = 4.5f * cpc - 1.5f * t.trp;
    if constexpr (ORDER >= 3) {
        eq += 4.5f * cu * (cu * cu - t.u2);
        neq += cu * (13.5f * cpc - 4.5f * t.trp) - 9.0f * (X * t.pux + Y * t.puy);
    }
    return W * (t.dr + t.rho * eq + t.omo * neq + 3.0f * (X * t.rgx + Y * t.rgy));
}

__device__ __forceinline__ float from_lane(int src_lane, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

template <class S>
__device__ __forceinline__ void load6(const typename S::T* __restrict__ st, long long N, long long n,
                                      const StepParams& p, float m[6]) {
    m[0] = S::load(st[n], p.inv_scale[0]);
    m[1] = S::load(st[1 * N + n], p.inv_scale[1]);
    m[2] = S::load(st[2 * N + n], p.inv_scale[1]);
    m[3] = S::load(st[4 * N + n], p.inv_scale[2]);
    m[4] = S::load(st[5 * N + n], p.inv_scale[2]);
    m[5] = S::load(st[7 * N + n], p.inv_scale[2]);
}

__device__ __forceinline__ int wrap_clamp(int v, int n, bool periodic) {
    if (periodic) {
        v %= n;
        return v < 0 ? v + n : v;
    }
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

template <class S, int ORDER, bool FIELD>
__global__ void __launch_bounds__(kD2Block) update_d2q9_kernel(const typename S::T* __restrict__ in,
                                                               typename S::T* __restrict__ out, StepParams p,
                                                               int strips, int segments, int seg_rows) {
    const Geometry& g = p.geo;
    const int nx = g.n[0], ny = g.n[1];
    const long long N = g.N;
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * (kD2Block / 64) + (threadIdx.x >> 6);
    if (item >= strips * segments) return;  // whole wavefronts leave together
    const int strip = item % strips, seg = item / strips;
    const int y0 = seg * seg_rows, y1 = min(y0 + seg_rows, ny);
    const int gx = strip * kStrip - 1 + lane;
    const bool px = (g.periodic & 1) != 0, py = (g.periodic & 2) != 0;
    const int x = wrap_clamp(gx, nx, px);
    const bool interior = lane >= 1 && lane <= kStrip && gx < nx;
    const bool col_solid = (x == 0 && (g.lo_solid & 1)) || (x == nx - 1 && (g.hi_solid & 1));
    const float omo = omo_at(p, 0);

    auto row = [&](int yp, Sums2& aprev, Sums2& acur, Sums2& anext) {
        const int y = wrap_clamp(yp, ny, py);
        const long long n = x + (long long)nx * y;
        float m[6];
        load6<S>(in, N, n, p, m);
        const bool solid = col_solid || (y == 0 && (g.lo_solid & 2)) || (y == ny - 1 && (g.hi_solid & 2));
        float gxv = 0.0f, gyv = 0.0f;
        if (!solid) {
            gxv = FIELD ? p.gfield[n] : p.force[0];
            gyv = FIELD ? p.gfield[N + n] : p.force[1];
        }
        const Terms2 t = terms2(m, gxv, gyv, omo);
        float G[9];
        G[0] = emit9<0, ORDER>(t);
        G[1] = emit9<1, ORDER>(t);
        G[2] = emit9<2, ORDER>(t);
        G[3] = emit9<3, ORDER>(t);
        G[4] = emit9<4, ORDER>(t);
        G[5] = emit9<5, ORDER>(t);
        G[6] = emit9<6, ORDER>(t);
        G[7] = emit9<7, ORDER>(t);
        G[8] = emit9<8, ORDER>(t);
        // arrivals at this lane: the population with c_x = +1 comes from the
        // lane on the left, c_x = -1 from the lane on the right
        const int left = (lane + 63) & 63, right = (lane + 1) & 63;
        // slice c_y = -1 (I = 0, 1, 2) arrives in row yp - 1
        aprev.template add<-1, -1>(from_lane(right, G[0]));
        aprev.template add<0, -1>(G[1]);
        aprev.template add<1, -1>(from_lane(left, G[2]));
        // slice c_y = 0 (I = 3, 4, 5) stays in row yp
        acur.template add<-1, 0>(from_lane(right, G[3]));
        acur.template add<0, 0>(G[4]);
        acur.template add<1, 0>(from_lane(left, G[5]));
        // slice c_y = +1 (I = 6, 7, 8) starts row yp + 1
        anext.zero();
        anext.template add<-1, 1>(from_lane(right, G[6]));
        anext.template add<0, 1>(G[7]);
        anext.template add<1, 1>(from_lane(left, G[8]));

        const int yo = yp - 1;  // row yp - 1 is complete
        if (!(interior && yo >= y0 && yo < y1)) return;
        const bool fluid_col = !col_solid && !(x == 0 && (g.lo_ghost & 1)) && !(x == nx - 1 && (g.hi_ghost & 1));
        const bool fluid = fluid_col && !(yo == 0 && ((g.lo_solid | g.lo_ghost) & 2)) &&
                           !(yo == ny - 1 && ((g.hi_solid | g.hi_ghost) & 2));
        if (!fluid) return;
        Sums2 a = aprev;
        // half-way bounce-back: for every c whose upstream node x - c is a
        // wall, the node's own population along -c arrives along c
        const bool wl = (g.lo_solid & 1) && x == 1, wr = (g.hi_solid & 1) && x == nx - 2;
        const bool wb = (g.lo_solid & 2) && yo == 1, wt = (g.hi_solid & 2) && yo == ny - 2;
        const long long no = x + (long long)nx * yo;
        if (wl || wr || wb || wt) {
            float mo[6];
            load6<S>(in, N, no, p, mo);
            const float ogx = FIELD ? p.gfield[no] : p.force[0];
            const float ogy = FIELD ? p.gfield[N + no] : p.force[1];
            const Terms2 to = terms2(mo, ogx, ogy, omo);
            // upstream of c = (X, Y) is (x - X, yo - Y)
#define TSLB_BB(I, X, Y)                                                        \
    if ((X == 1 && wl) || (X == -1 && wr) || (Y == 1 && wb) || (Y == -1 && wt)) \
        a.template add<X, Y>(emit9<8 - I, ORDER>(to));
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
        // drho' = D/36, u' = J/(36 + D), Pi' = (S - J u' - D/3 delta)/36
        const float den = 36.0f + a.d;
        float inv = __builtin_amdgcn_rcpf(den);
        inv = inv * fmaf(-den, inv, 2.0f);
        const float ux = a.jx * inv, uy = a.jy * inv, d3 = a.d * (1.0f / 3.0f);
        constexpr float k36 = 1.0f / 36.0f;
        out[no] = S::store(a.d * k36, p.scale[0]);
        out[1 * N + no] = S::store(ux, p.scale[1]);
        out[2 * N + no] = S::store(uy, p.scale[1]);
        out[4 * N + no] = S::store((a.sxx - a.jx * ux - d3) * k36, p.scale[2]);
        out[5 * N + no] = S::store((a.syy - a.jy * uy - d3) * k36, p.scale[2]);
        out[7 * N + no] = S::store((a.sxy - a.jx * uy) * k36, p.scale[2]);
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
    const int waves = strips * segments;
    const unsigned grid = (unsigned)((waves + kD2Block / 64 - 1) / (kD2Block / 64));
    if (p.gfield)
        hipLaunchKernelGGL((update_d2q9_kernel<S, ORDER, true>), dim3(grid), dim3(kD2Block), 0, s,
                           (const typename S::T*)in, (typename S::T*)out, p, strips, segments, seg_rows);
    else
        hipLaunchKernelGGL((update_d2q9_kernel<S, ORDER, false>), dim3(grid), dim3(kD2Block), 0, s,
                           (const typename S::T*)in, (typename S::T*)out, p, strips, segments, seg_rows);
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
    if (p.geo.n[2] != 1) return hipErrorInvalidValue;
    const int strips = (nx + kStrip - 1) / kStrip;
    // rows per segment: enough wavefronts to fill the chip (about 16 per CU)
    // while keeping the two halo rows of a segment a small overhead
    const long long target = 256LL * 16;
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
