// Device-side building blocks of the gfx950 TSLB kernels: grid geometry,
// moment storage formats, the D3Q27 velocity set and the per-population
// reconstruction of the thread-safe update (Montessori et al.,
// arXiv:2401.17074, Section 2.2).
//
// Arithmetic form.  With c_s^2 = 1/3 the population a node with moments
// (rho, u, Pi) emits along c is w(c) (1 + P(c)), where the deviation
//   P(c) = drho + rho [3 cu + 9/2 cu^2 - 3/2 u^2 + 9/2 cu (cu^2 - u^2)]
//        + (1 - omega) [9/2 (cPc - tr Pi / 3) + 27/2 cPc cu - 9/2 tr Pi cu
//                       - 9 c.(Pi u)]  + 3 rho c.g
// is the Hermite equilibrium of Eq. (eqts) minus its rest value plus the
// recursive non-equilibrium part of Eq. (noneqts) and the local forcing of
// Section 3.1, expanded with H2 = cc - 1/3, H3 contracted on u u u and on the
// symmetrised a3 = Pi u.  Only drho = rho - 1 and the deviations are summed,
// never 1 + small, which keeps FP32 round-off at the level of the
// fluctuations.
//
// Exact weights.  The D3Q27 weights are (1/216) 4^n0 with n0 the number of
// zero components of c, so the kernels carry G = 216 w P = 4^n0 P (an exact
// power-of-two scaling) and apply 1/216 once per stored moment.  Binary32
// roundings of 2/3 and 1/6 would otherwise perturb the lattice itself (its
// isotropy sums) by ~1e-7 every step, a bias that accumulates coherently.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace tslb {

// ------------------------------------------------------------------ geometry
enum FaceKind { kPeriodic = 0, kWall = 1, kInlet = 2, kOutlet = 3 };

struct Geometry {
    int n[3];          // nx, ny, nz
    long long N;       // nx * ny * nz
    int periodic;      // bit d: axis d periodic
    int lo_solid;      // bit d: layer 0 of axis d is a wall
    int hi_solid;      // bit d: layer n_d - 1 of axis d is a wall
    int lo_ghost;      // bit d: layer 0 of axis d is an inflow/outflow ghost layer
    int hi_ghost;      // bit d: layer n_d - 1 is a ghost layer
};

__device__ __forceinline__ bool is_solid(const Geometry& g, int x, int y, int z) {
    int c[3] = {x, y, z};
    bool s = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s |= (c[d] == 0) && ((g.lo_solid >> d) & 1);
        s |= (c[d] == g.n[d] - 1) && ((g.hi_solid >> d) & 1);
    }
    return s;
}

__device__ __forceinline__ bool is_fluid(const Geometry& g, int x, int y, int z) {
    int c[3] = {x, y, z};
    bool f = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        f &= !((c[d] == 0) && (((g.lo_solid | g.lo_ghost) >> d) & 1));
        f &= !((c[d] == g.n[d] - 1) && (((g.hi_solid | g.hi_ghost) >> d) & 1));
    }
    return f;
}

// Wall face next to a fluid node (the first of -x, +x, -y, +y, -z, +z whose
// wall layer is a neighbour), or -1.  Faces: bit d of lo_solid / hi_solid.
__device__ __forceinline__ int first_wall_face(const Geometry& g, const int c[3]) {
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1;
        const bool wall = (f & 1) ? ((g.hi_solid >> d) & 1) : ((g.lo_solid >> d) & 1);
        const int layer = (f & 1) ? g.n[d] - 2 : 1;
        if (wall && c[d] == layer) return f;
    }
    return -1;
}

// Position of a node inside the layer of face f: the two transverse
// coordinates (in x, y, z order) as a + n_a * b.
__device__ __forceinline__ long long wall_layer_index(const Geometry& g, int f, const int c[3]) {
    const int d = f >> 1;
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    return (long long)c[d1] + (long long)g.n[d1] * c[d2];
}

// ------------------------------------------------------------------ storage
// Stored field q of a node: FP32 as is; FP16 / BF16 hold value * scale[q]
// rounded to nearest even.  Field 0 holds rho - 1.
// convert / pack are the plain format conversions, load / store add the
// field's scale (exact: the scales are powers of two).
struct StoreF32 {
    using T = float;
    __device__ __forceinline__ static float convert(T v) { return v; }
    __device__ __forceinline__ static T pack(float v) { return v; }
    __device__ __forceinline__ static float load(T v, float) { return v; }
    __device__ __forceinline__ static T store(float v, float) { return v; }
};

struct StoreF16 {
    using T = __half;
    __device__ __forceinline__ static float convert(T v) { return __half2float(v); }
    __device__ __forceinline__ static T pack(float v) { return __float2half_rn(v); }
    __device__ __forceinline__ static float load(T v, float inv_scale) { return convert(v) * inv_scale; }
    __device__ __forceinline__ static T store(float v, float scale) { return pack(v * scale); }
};

// bfloat16 kept as raw 16-bit patterns: the upper half of a binary32 after
// round-to-nearest-even on the dropped 16 bits (NaN stays NaN), which is
// gfx950's own float-to-bfloat16 conversion (one instruction).
struct StoreBF16 {
    using T = uint16_t;
    __device__ __forceinline__ static float convert(T v) { return __uint_as_float(((uint32_t)v) << 16); }
    __device__ __forceinline__ static T pack(float v) { return __builtin_bit_cast(T, static_cast<__bf16>(v)); }
    __device__ __forceinline__ static float load(T v, float inv_scale) { return convert(v) * inv_scale; }
    __device__ __forceinline__ static T store(float v, float scale) { return pack(v * scale); }
};

// ------------------------------------------------------------------ lattice
// The 27 velocities ordered i = 9 (cz + 1) + 3 (cy + 1) + (cx + 1), so the
// opposite of i is 26 - i.  The weight of i is w216_of(i) / 216 with
// w216 = 4^(number of zero components): 64, 16, 4, 1 for the rest, face,
// edge and corner velocities.
__host__ __device__ constexpr int cx_of(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz_of(int i) { return i / 9 - 1; }
__host__ __device__ constexpr float w216_of(int i) {
    return (float)(1 << (2 * ((cx_of(i) == 0) + (cy_of(i) == 0) + (cz_of(i) == 0))));
}
constexpr float kInv216 = 1.0f / 216.0f;

// Per-node quantities the 27 reconstructions share.
struct NodeTerms {
    float drho, rho;
    float u[3];
    float u2;          // |u|^2
    float p[6];        // Pi xx, yy, zz, xy, xz, yz
    float trp;         // tr Pi
    float pu[3];       // Pi u
    float rg[3];       // rho g
};

__device__ __forceinline__ NodeTerms node_terms(const float m[10], const float g[3]) {
    NodeTerms t;
    t.drho = m[0];
    t.rho = 1.0f + m[0];
    t.u[0] = m[1];
    t.u[1] = m[2];
    t.u[2] = m[3];
    t.u2 = m[1] * m[1] + m[2] * m[2] + m[3] * m[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) t.p[k] = m[4 + k];
    t.trp = m[4] + m[5] + m[6];
    t.pu[0] = m[4] * m[1] + m[7] * m[2] + m[8] * m[3];
    t.pu[1] = m[7] * m[1] + m[5] * m[2] + m[9] * m[3];
    t.pu[2] = m[8] * m[1] + m[9] * m[2] + m[6] * m[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) t.rg[a] = t.rho * g[a];
    return t;
}

// Scaled deviation G = 216 w(c) P(c) of the population emitted along
// velocity I (compile-time).  ORDER 2 drops the third-order Hermite terms of
// both parts (the regularised collision of Eq. (fullstrcoll)).
template <int I, int ORDER = 3>
__device__ __forceinline__ float emit_dev(const NodeTerms& t, float one_minus_omega) {
    constexpr int X = cx_of(I), Y = cy_of(I), Z = cz_of(I);
    constexpr float W = w216_of(I);
    const float cu = X * t.u[0] + Y * t.u[1] + Z * t.u[2];
    const float cpc = X * X * t.p[0] + Y * Y * t.p[1] + Z * Z * t.p[2] +
                      2.0f * (X * Y * t.p[3] + X * Z * t.p[4] + Y * Z * t.p[5]);
    const float cpu = X * t.pu[0] + Y * t.pu[1] + Z * t.pu[2];
    const float cg = X * t.rg[0] + Y * t.rg[1] + Z * t.rg[2];
    float eq = cu * (3.0f + 4.5f * cu) - 1.5f * t.u2;
    float neq = 4.5f * cpc - 1.5f * t.trp;
    if constexpr (ORDER >= 3) {
        eq += 4.5f * cu * (cu * cu - t.u2);
        neq += cu * (13.5f * cpc - 4.5f * t.trp) - 9.0f * cpu;
    }
    return W * (t.drho + t.rho * eq + one_minus_omega * neq + 3.0f * cg);
}

// Moment accumulators of the arriving scaled deviations G = 216 w P:
// D = sum G, J = sum G c, S = sum G c c (xx, yy, zz, xy, xz, yz).
struct MomentSums {
    float d, j[3], s[6];
    __device__ __forceinline__ void zero() {
        d = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) j[a] = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] = 0.f;
    }
    template <int I>
    __device__ __forceinline__ void add(float f) {
        constexpr int X = cx_of(I), Y = cy_of(I), Z = cz_of(I);
        d += f;
        if (X) j[0] += X * f;
        if (Y) j[1] += Y * f;
        if (Z) j[2] += Z * f;
        if (X) s[0] += f;
        if (Y) s[1] += f;
        if (Z) s[2] += f;
        if (X * Y) s[3] += X * Y * f;
        if (X * Z) s[4] += X * Z * f;
        if (Y * Z) s[5] += Y * Z * f;
    }
};

// New moments from the summed scaled deviations (Section 2: rho = sum f,
// rho u = sum f c, Pi^neq = sum f c c - rho u u - rho/3 delta).  With
// sum f = 1 + D/216, sum f c = J/216 and sum f c c = delta/3 + S/216:
//   drho' = D/216,  u' = J / (216 + D),
//   Pi'   = (S - J u' - D/3 delta) / 216.
// SCALE is the exact factor the populations carry: 216 for the D3Q27
// weights (216 w = 4^n0), 36 for D3Q19 (36 w = 12, 2, 1 for the rest, face
// and edge velocities).
template <int SCALE = 216>
__device__ __forceinline__ void finalize(const MomentSums& a, float out[10]) {
    constexpr float kInv = 1.0f / (float)SCALE;
    // 1 / (SCALE + D): hardware reciprocal refined by one Newton step
    const float den = (float)SCALE + a.d;
    float inv = __builtin_amdgcn_rcpf(den);
    inv = inv * fmaf(-den, inv, 2.0f);
    const float ux = a.j[0] * inv, uy = a.j[1] * inv, uz = a.j[2] * inv;
    const float d3 = a.d * (1.0f / 3.0f);
    out[0] = a.d * kInv;
    out[1] = ux;
    out[2] = uy;
    out[3] = uz;
    out[4] = (a.s[0] - a.j[0] * ux - d3) * kInv;
    out[5] = (a.s[1] - a.j[1] * uy - d3) * kInv;
    out[6] = (a.s[2] - a.j[2] * uz - d3) * kInv;
    out[7] = (a.s[3] - a.j[0] * uy) * kInv;
    out[8] = (a.s[4] - a.j[0] * uz) * kInv;
    out[9] = (a.s[5] - a.j[1] * uz) * kInv;
}

// finalize() with the stored fields' scales s0 (drho), s1 (u), s2 (Pi)
// applied: folded into the 1/SCALE factor where there is one (the same
// values, since the scales are powers of two).
template <int SCALE = 216>
__device__ __forceinline__ void finalize_scaled(const MomentSums& a, float s0, float s1, float s2, float out[10]) {
    constexpr float kInv = 1.0f / (float)SCALE;
    const float k0 = kInv * s0, k2 = kInv * s2;
    const float den = (float)SCALE + a.d;
    float inv = __builtin_amdgcn_rcpf(den);
    inv = inv * fmaf(-den, inv, 2.0f);
    const float ux = a.j[0] * inv, uy = a.j[1] * inv, uz = a.j[2] * inv;
    const float d3 = a.d * (1.0f / 3.0f);
    out[0] = a.d * k0;
    out[1] = ux * s1;
    out[2] = uy * s1;
    out[3] = uz * s1;
    out[4] = (a.s[0] - a.j[0] * ux - d3) * k2;
    out[5] = (a.s[1] - a.j[1] * uy - d3) * k2;
    out[6] = (a.s[2] - a.j[2] * uz - d3) * k2;
    out[7] = (a.s[3] - a.j[0] * uy) * k2;
    out[8] = (a.s[4] - a.j[0] * uz) * k2;
    out[9] = (a.s[5] - a.j[1] * uz) * k2;
}

// Compile-time loop over the 27 velocities.
template <int I, int END>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void run(F&& f) {
        f.template operator()<I>();
        Unroll<I + 1, END>::run(f);
    }
};
template <int END>
struct Unroll<END, END> {
    template <class F>
    __device__ __forceinline__ static void run(F&&) {}
};

}  // namespace tslb
