// Tiled discrete adjoint of the update for gfx950: the exact transpose of the
// tiled forward kernel.
//
// Forward: node y emits f_i(y) = w_i P_y(c_i) (P polynomial in c with the 17
// coefficients A_k(M_y, g_y)) to x = y + c_i, and x sums what arrives into
// its new moments M'(x).  Reverse, for a sensitivity lam' = dL/dM'(x):
//   a_x(c) = dL/df_i at x = lam'_rho + lam'_u.(c - u')/rho'
//            + lam'_Pi : [(c - u')(c - u') - delta/3]
// is a quadratic in c (10 coefficients), so every node x evaluates its 27
// arrival sensitivities once and publishes them in LDS; every source node y
// gathers a_{y+c_i}(c_i) from its downstream neighbours, forms the 17
// weighted monomial moments Lambda_k = sum_i w_i m_k(c_i) a_{y+c_i}(c_i), and
// pulls them back through the coefficient map (coefficients_vjp).  Wall
// nodes carry zero sensitivity; a node whose upstream node along c_j is a
// wall received its own population along -c_j there, so a_y(c_j) is added
// as a value arriving along -c_j (done in the same pass for the few lanes
// next to a wall).
#include "tslb_tiles.h"

namespace tslb {
namespace {

using namespace tile;

// arrival-sensitivity coefficients, order: 1, cx, cy, cz, cx^2, cy^2, cz^2,
// cx cy, cx cz, cy cz
__host__ __device__ inline void arrival_coefficients(const float lam[10], float drho1, const float u[3], float B[10]) {
    const float q = 1.0f / (1.0f + drho1);
    const float ux = u[0], uy = u[1], uz = u[2];
    const float third = 1.0f / 3.0f;
    B[4] = lam[4];
    B[5] = lam[5];
    B[6] = lam[6];
    B[7] = lam[7];
    B[8] = lam[8];
    B[9] = lam[9];
    B[1] = lam[1] * q - 2.0f * lam[4] * ux - lam[7] * uy - lam[8] * uz;
    B[2] = lam[2] * q - 2.0f * lam[5] * uy - lam[7] * ux - lam[9] * uz;
    B[3] = lam[3] * q - 2.0f * lam[6] * uz - lam[8] * ux - lam[9] * uy;
    B[0] = lam[0] - q * (lam[1] * ux + lam[2] * uy + lam[3] * uz) + lam[4] * (ux * ux - third) +
           lam[5] * (uy * uy - third) + lam[6] * (uz * uz - third) + lam[7] * ux * uy + lam[8] * ux * uz +
           lam[9] * uy * uz;
}

// 216 w(c) a(c) on the 27 velocities (same separable scheme as the
// populations: per cz slice a quadratic in (cx, cy)).
__device__ __forceinline__ void arrival_values(const float B[10], float G[27]) {
    eval_slice<0>(B[0], B[1], B[2], B[4], B[5], B[7], 0.0f, 0.0f, G);
    const float e0 = B[0] + B[6];
    eval_slice<1>(e0 + B[3], B[1] + B[8], B[2] + B[9], B[4], B[5], B[7], 0.0f, 0.0f, G);
    eval_slice<-1>(e0 - B[3], B[1] - B[8], B[2] - B[9], B[4], B[5], B[7], 0.0f, 0.0f, G);
}

// the 17 weighted monomial moments of the values gathered for one node
struct AdjSums {
    float L[NK];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < NK; ++k) L[k] = 0.0f;
    }
};

// One cz slice F[cy+1][cx+1] (216 w a values) added to the monomial moments:
// sum F cx^a cy^b cz^c for every monomial (a, b, c) of the coefficient map.
template <int CZ>
__device__ __forceinline__ void add_adj_slice(const float F[3][3], AdjSums& a) {
    float s[3], d[3], t[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        s[r] = F[r][0] + F[r][2];
        d[r] = F[r][2] - F[r][0];
        t[r] = s[r] + F[r][1];
    }
    const float m02 = t[2] + t[0], m00 = m02 + t[1], m01 = t[2] - t[0];
    const float m12 = d[2] + d[0], m10 = m12 + d[1], m11 = d[2] - d[0];
    const float m20 = s[0] + s[1] + s[2], m21 = s[2] - s[0];
    a.L[K000] += m00;
    a.L[K100] += m10;
    a.L[K010] += m01;
    a.L[K200] += m20;
    a.L[K020] += m02;
    a.L[K110] += m11;
    a.L[K210] += m21;
    a.L[K120] += m12;
    if (CZ != 0) {
        a.L[K001] += CZ * m00;
        a.L[K101] += CZ * m10;
        a.L[K011] += CZ * m01;
        a.L[K201] += CZ * m20;
        a.L[K021] += CZ * m02;
        a.L[K111] += CZ * m11;
        a.L[K002] += m00;
        a.L[K102] += m10;
        a.L[K012] += m01;
    }
}


// The adjoint runs one block per tile (on grids small enough to be bound by
// latency, such as the 64^3 box of the gradient workload, this is faster
// than walking the update's work list, which costs a dependent load before
// the first address).  Planes per tile: every block costs about (tz + 2)
// plane-steps and the blocks run in rounds of one per CU, so take the tz in
// [1, 64] that minimises rounds x (tz + 2).
inline int choose_tz(int columns, int nz, int cus) {
    int best = 32;
    long long best_cost = -1;
    for (int tz = 1; tz <= 64; ++tz) {
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
// Consecutive block ids are dealt round-robin to the 8 XCDs: block b takes
// tile (b % 8) * ceil(nblk / 8) + b / 8, so each XCD gets a contiguous run of
// neighbouring tiles; padding blocks (the grid is a multiple of 8) get -1.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
    const int per = (nblk + 7) >> 3;
    const int t = (b & 7) * per + (b >> 3);
    return t < nblk ? t : -1;
}
inline unsigned xcd_grid(int nblk) { return (unsigned)((nblk + 7) & ~7); }

template <bool WALLS, bool FIELD, bool DG>
__global__ void __launch_bounds__(NTHREADS, TSLB_WAVES_PER_EU)
    adjoint_tiled_kernel(const float* __restrict__ st0, const float* __restrict__ st1, const float* __restrict__ lam1,
                         float* __restrict__ lam0, float* __restrict__ dg, StepParams p, int tiles_x, int tiles_y,
                         int tiles_z, int TZ) {
    __shared__ float lds[NSLOT][LY][LX];
    const Geometry& g = p.geo;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned long long N = (unsigned long long)g.N;
    const unsigned plane_nodes = (unsigned)nx * (unsigned)ny;

    const int b = xcd_tile(blockIdx.x, tiles_x * tiles_y * tiles_z);
    if (b < 0) return;  // padding block (before any barrier)
    const int tx = b % tiles_x;
    const int ty = (b / tiles_x) % tiles_y;
    const int tz = b / (tiles_x * tiles_y);
    const int x0 = tx * TX, y0 = ty * TY;
    const int zs = tz * TZ;
    const int ze = min(zs + TZ, nz);

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
    const bool valid = interior && gx < nx && gy < ny;
    // only fluid nodes carry sensitivity (walls never pull populations)
    const bool col_fluid_any = !((wx == 0 && (g.lo_solid & 1)) || (wx == nx - 1 && (g.hi_solid & 1)) ||
                                 (wy == 0 && (g.lo_solid & 2)) || (wy == ny - 1 && (g.hi_solid & 2)));
    const int wf = (WALLS && interior) ? wall_flags(g, gx, gy) : 0;
    const bool zlo_wall = (g.lo_solid & 4) != 0, zhi_wall = (g.hi_solid & 4) != 0;

    // arrival sensitivities of node (col, zp) into G
    auto arrivals = [&](int zp, float G[27]) {
        const unsigned n = col + plane_nodes * (unsigned)plane_index(zp, nz, pz);
        const bool plane_wall = (zlo_wall && plane_index(zp, nz, pz) == 0) ||
                                (zhi_wall && plane_index(zp, nz, pz) == nz - 1);
        const float on = (col_fluid_any && !plane_wall) ? 1.0f : 0.0f;
        float l[10], u1[3];
#pragma unroll
        for (int k = 0; k < 10; ++k) l[k] = on * lam1[k * N + n];
        const float d1 = st1[n];
#pragma unroll
        for (int a = 0; a < 3; ++a) u1[a] = st1[(1 + a) * N + n];
        float B[10];
        arrival_coefficients(l, d1, u1, B);
        arrival_values(B, G);
    };

    // plane zp: publish its arrival sensitivities; what node (col, zp - cz)
    // gathers along direction (cx, cy, cz) is at (col + (cx, cy), zp): the
    // slice cz of plane zp goes to output plane zp - cz.
    auto plane = [&](int zp, AdjSums& aprev, AdjSums& acur, AdjSums& anext) {
        float G[27];
        if (active) {
            arrivals(zp, G);
            Unroll<0, 27>::run([&]<int I>() {
                if constexpr (cx_of(I) != 0 || cy_of(I) != 0) lds[slot_of(I)][ly][lx] = G[I];
            });
        }
        __syncthreads();
        if (interior) {
            auto gather_slice = [&]<int CZ>(float (&F)[3][3]) {
                Unroll<0, 9>::run([&]<int K>() {
                    constexpr int I = 9 * (CZ + 1) + K;
                    constexpr int X = cx_of(I), Y = cy_of(I);
                    if constexpr (X == 0 && Y == 0)
                        F[Y + 1][X + 1] = G[I];
                    else
                        F[Y + 1][X + 1] = lds[slot_of(I)][ly + Y][lx + X];
                });
            };
            float F[3][3];
            gather_slice.template operator()<1>(F);
            add_adj_slice<1>(F, aprev);
            gather_slice.template operator()<0>(F);
            add_adj_slice<0>(F, acur);
            gather_slice.template operator()<-1>(F);
            add_adj_slice<-1>(F, anext);
            if (WALLS) {
                // own population bounced back: a_y(c_j) arrives as if along -c_j
                const bool zlo = zlo_wall && zp == 1, zhi = zhi_wall && zp == nz - 2;
                // bounce-back happens at fluid nodes only (ghost nodes are
                // sources, never updated)
                if ((wf != 0 || zlo || zhi) && is_fluid(g, gx, gy, zp)) {
                    auto bounce_slice = [&]<int CZ>(float (&Fb)[3][3]) {
                        Unroll<0, 9>::run([&]<int K>() {
                            constexpr int I = 9 * (CZ + 1) + K, J = 26 - I;  // J = -c_I
                            float own;
                            if constexpr (cx_of(J) == 0 && cy_of(J) == 0)
                                own = G[J];
                            else
                                own = lds[slot_of(J)][ly][lx];
                            Fb[cy_of(I) + 1][cx_of(I) + 1] = upstream_solid<J>(wf, zlo, zhi) ? own : 0.0f;
                        });
                    };
                    bounce_slice.template operator()<-1>(F);
                    add_adj_slice<-1>(F, acur);
                    bounce_slice.template operator()<0>(F);
                    add_adj_slice<0>(F, acur);
                    bounce_slice.template operator()<1>(F);
                    add_adj_slice<1>(F, acur);
                }
            }
        }
        // output plane zp - 1 is complete
        const int zo = zp - 1;
        if (interior && zo >= zs && zo < ze && valid) {
            const unsigned on = col + plane_nodes * (unsigned)zo;
            // every node that emits (fluid or ghost; walls emit nothing)
            const bool fl = col_fluid_any && !(zlo_wall && zo == 0) && !(zhi_wall && zo == nz - 1) &&
                            !is_solid(g, gx, gy, zo);
            float out[10], lg[3] = {0.0f, 0.0f, 0.0f};
            float dg_old[3] = {0.0f, 0.0f, 0.0f};  // read with the moments, not after the stores
            if (fl) {
                float m[10], gg[3];
#pragma unroll
                for (int k = 0; k < 10; ++k) m[k] = st0[k * N + on];
#pragma unroll
                for (int a = 0; a < 3; ++a) gg[a] = FIELD ? p.gfield[a * N + on] : p.force[a];
                if (DG) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) dg_old[a] = dg[a * N + on];
                }
                float L[NK];
#pragma unroll
                for (int k = 0; k < NK; ++k) L[k] = aprev.L[k] * kInv216;
                coefficients_vjp(L, m, gg, omo_at(p, zo), out, lg);
            } else {
#pragma unroll
                for (int k = 0; k < 10; ++k) out[k] = 0.0f;
            }
#pragma unroll
            for (int k = 0; k < 10; ++k) lam0[k * N + on] = out[k];
            if (DG && fl) {
#pragma unroll
                for (int a = 0; a < 3; ++a) dg[a * N + on] = dg_old[a] + lg[a];
            }
        }
        aprev.zero();
        __syncthreads();
    };

    AdjSums a0, a1, a2;
    a0.zero();
    a1.zero();
    a2.zero();
    for (int zp = zs - 1; zp <= ze; zp += 3) {
        plane(zp, a0, a1, a2);
        if (zp + 1 > ze) break;
        plane(zp + 1, a1, a2, a0);
        if (zp + 2 > ze) break;
        plane(zp + 2, a2, a0, a1);
    }
}

template <bool WALLS, bool FIELD, bool DG>
hipError_t launch_t(const float* st0, const float* st1, const float* lam1, float* lam0, float* dg,
                    const StepParams& p, hipStream_t s) {
    const int tiles_x = (p.geo.n[0] + TX - 1) / TX;
    const int tiles_y = (p.geo.n[1] + TY - 1) / TY;
    const int TZ = choose_tz(tiles_x * tiles_y, p.geo.n[2], compute_units() * kBlocksPerCu);
    const int tiles_z = (p.geo.n[2] + TZ - 1) / TZ;
    const unsigned nblk = (unsigned)tiles_x * tiles_y * tiles_z;
    if (p.geo.N >= (1LL << 30)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((adjoint_tiled_kernel<WALLS, FIELD, DG>), dim3(xcd_grid(nblk)), dim3(NTHREADS), 0, s, st0, st1, lam1,
                       lam0, dg, p, tiles_x, tiles_y, tiles_z, TZ);
    return hipGetLastError();
}

template <bool WALLS>
hipError_t launch_w(const float* st0, const float* st1, const float* lam1, float* lam0, float* dg,
                    const StepParams& p, hipStream_t s) {
    const bool field = p.gfield != nullptr;
    if (dg)
        return field ? launch_t<WALLS, true, true>(st0, st1, lam1, lam0, dg, p, s)
                     : launch_t<WALLS, false, true>(st0, st1, lam1, lam0, dg, p, s);
    return field ? launch_t<WALLS, true, false>(st0, st1, lam1, lam0, dg, p, s)
                 : launch_t<WALLS, false, false>(st0, st1, lam1, lam0, dg, p, s);
}

}  // namespace

hipError_t launch_adjoint_tiled(const float* st0, const float* st1, const float* lam1, float* lam0, float* dg,
                                const StepParams& p, hipStream_t s) {
    if ((p.geo.lo_solid | p.geo.hi_solid) != 0) return launch_w<true>(st0, st1, lam1, lam0, dg, p, s);
    return launch_w<false>(st0, st1, lam1, lam0, dg, p, s);
}

}  // namespace tslb
