// Kernels around the update: ghost-layer refill (Section 2.3), conversion
// between caller arrays and the stored format, FP64 reductions, and the
// discrete adjoint of one update step.
#include "tslb_internal.h"

namespace tslb {
namespace {

// ---------------------------------------------------------------- ghosts
// Threads enumerate the six face layers one after the other; a node shared
// by several ghost faces is written once (by its lowest ghost face).  Each
// ghost node takes the ten stored values of its interior neighbour
// (coordinates clamped into the interior along every ghost axis); nodes of
// an inlet disc then get the imposed velocity with the seeded perturbation.
//
// With x_done set the tiled update has already written the ghost nodes of
// the x faces that lie on no other ghost face (each from the interior node
// next to it, the value it had just computed): those only get the inlet
// velocity where it applies.
template <class S>
__global__ void ghost_fill_kernel(typename S::T* __restrict__ st, StepParams p, InletParams q, int64_t t,
                                  long long off1, long long off2, long long off3, long long off4,
                                  long long off5, long long total, int x_done) {
    const Geometry& g = p.geo;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= total) return;
    const long long offs[6] = {0, off1, off2, off3, off4, off5};
    int f = 5;
    while (f > 0 && tid < offs[f]) --f;
    if (q.face_kind[f] != kInlet && q.face_kind[f] != kOutlet) return;
    const int d = f >> 1;
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    const long long local = tid - offs[f];
    int c[3];
    c[d] = face_layer(g, f);
    c[d1] = (int)(local % g.n[d1]);
    c[d2] = (int)(local / g.n[d1]);
    if (c[d2] >= g.n[d2]) return;
    if (is_solid(g, c[0], c[1], c[2])) return;
    for (int f2 = 0; f2 < f; ++f2)
        if ((q.face_kind[f2] == kInlet || q.face_kind[f2] == kOutlet) && c[f2 >> 1] == face_layer(g, f2)) return;
    int cf[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cf[a] = c[a];
        if (c[a] == 0 && ((g.lo_ghost >> a) & 1)) cf[a] = 1;
        if (c[a] == g.n[a] - 1 && ((g.hi_ghost >> a) & 1)) cf[a] = g.n[a] - 2;
    }
    const long long n = c[0] + (long long)g.n[0] * (c[1] + (long long)g.n[1] * c[2]);
    const long long nf = cf[0] + (long long)g.n[0] * (cf[1] + (long long)g.n[1] * cf[2]);
    float u[3];
    if (x_done && d == 0 && cf[1] == c[1] && cf[2] == c[2]) {
        if (inlet_velocity(g, q, p.dims, t, n, c, u))
            for (int a = 0; a < p.dims; ++a) st[(1 + a) * g.N + n] = S::store(u[a], p.scale[1]);
        return;
    }
    // all ten loads first: the source is an interior node this kernel never
    // writes, and one wait replaces ten load-store round trips
    typename S::T v[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) v[k] = st[k * g.N + nf];
#pragma unroll
    for (int k = 0; k < 10; ++k) st[k * g.N + n] = v[k];
    if (inlet_velocity(g, q, p.dims, t, n, c, u))
        for (int a = 0; a < p.dims; ++a) st[(1 + a) * g.N + n] = S::store(u[a], p.scale[1]);
}

// ---------------------------------------------------------------- pack/unpack
template <class S>
__global__ void pack_kernel(const float* __restrict__ rho, const float* __restrict__ u, const float* __restrict__ pi,
                            int rho_dev, typename S::T* __restrict__ st, StepParams p) {
    const Geometry& g = p.geo;
    const long long N = g.N;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    // wall nodes hold the zero deviation (rest state): the tiled update
    // relies on them emitting nothing
    const int x = (int)(n % g.n[0]);
    const int y = (int)((n / g.n[0]) % g.n[1]);
    const int z = (int)(n / ((long long)g.n[0] * g.n[1]));
    const float keep = is_solid(g, x, y, z) ? 0.0f : 1.0f;
    const float r = rho[n];
    st[n] = S::store(keep * (rho_dev ? r : r - 1.0f), p.scale[0]);
    // a two-dimensional lattice keeps u_z and the Pi components with a z
    // index (zz, xz, yz) at zero
    const float kz = p.dims == 2 ? 0.0f : keep;
#pragma unroll
    for (int a = 0; a < 3; ++a) st[(1 + a) * N + n] = S::store((a == 2 ? kz : keep) * u[a * N + n], p.scale[1]);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float kk = (k == 2 || k == 4 || k == 5) ? kz : keep;
        st[(4 + k) * N + n] = S::store(pi ? kk * pi[k * N + n] : 0.0f, p.scale[2]);
    }
}

template <class S>
__global__ void unpack_kernel(const typename S::T* __restrict__ st, float* __restrict__ rho, float* __restrict__ u,
                              float* __restrict__ pi, int rho_dev, StepParams p) {
    const long long N = p.geo.N;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    if (rho) {
        const float d = S::load(st[n], p.inv_scale[0]);
        rho[n] = rho_dev ? d : 1.0f + d;
    }
    if (u)
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a * N + n] = S::load(st[(1 + a) * N + n], p.inv_scale[1]);
    if (pi)
#pragma unroll
        for (int k = 0; k < 6; ++k) pi[k * N + n] = S::load(st[(4 + k) * N + n], p.inv_scale[2]);
}

// Weight of Pi_xd (d = 1: y, d = 2: z) in the wall shear objective at a
// fluid node: the x force on the walls normal to axis d, sum of s_f sigma_xd
// over the wall faces f the node is next to, with sigma = -(1 - omega/2) Pi
// and s_f = +1 (low face) or -1 (high face).  1 - omega/2 = (1 + (1 - omega))/2.
__device__ __forceinline__ double wall_shear_weight(const Geometry& g, const StepParams& p, int y, int z, int d) {
    const int c = d == 1 ? y : z;
    const double k = 0.5 * (1.0 + (double)omo_at(p, z));
    double w = 0.0;
    if (((g.lo_solid >> d) & 1) && c == 1) w -= k;
    if (((g.hi_solid >> d) & 1) && c == g.n[d] - 2) w += k;
    return w;
}

// ---------------------------------------------------------------- reductions
// Two passes with a fixed order, so the FP64 sums are reproducible.
constexpr int kRedThreads = 256;

template <class S>
__global__ void __launch_bounds__(kRedThreads) reduce_partial_kernel(const typename S::T* __restrict__ st,
                                                                     double* __restrict__ partials, StepParams p) {
    const Geometry& g = p.geo;
    double acc[kRedSums] = {0, 0, 0, 0, 0, 0, 0};
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < g.N;
         n += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(n % g.n[0]);
        const int y = (int)((n / g.n[0]) % g.n[1]);
        const int z = (int)(n / ((long long)g.n[0] * g.n[1]));
        if (!is_fluid(g, x, y, z)) continue;
        float m[10];
        m[0] = S::load(st[n], p.inv_scale[0]);
        for (int q = 1; q < 4; ++q) m[q] = S::load(st[q * g.N + n], p.inv_scale[1]);
        for (int q = 4; q < 10; ++q) m[q] = S::load(st[q * g.N + n], p.inv_scale[2]);
        bool bad = false;
        for (int q = 0; q < 10; ++q) bad |= !isfinite(m[q]);
        const double rho = 1.0 + (double)m[0];
        const double ux = m[1], uy = m[2], uz = m[3];
        acc[0] += rho;
        acc[1] += rho * ux;
        acc[2] += rho * uy;
        acc[3] += rho * uz;
        acc[4] += 0.5 * rho * (ux * ux + uy * uy + uz * uz);
        acc[5] += bad ? 1.0 : 0.0;
        acc[6] += wall_shear_weight(g, p, y, z, 1) * (double)m[7] + wall_shear_weight(g, p, y, z, 2) * (double)m[8];
    }
    __shared__ double sh[kRedSums][kRedThreads];
    for (int k = 0; k < kRedSums; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < kRedSums; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < kRedSums; ++k) partials[k * gridDim.x + blockIdx.x] = sh[k][0];
}

__global__ void __launch_bounds__(kRedThreads) reduce_final_kernel(const double* __restrict__ partials, int nblocks,
                                                                   double* __restrict__ out6) {
    __shared__ double sh[kRedThreads];
    for (int k = 0; k < kRedSums; ++k) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) a += partials[k * nblocks + b];
        sh[threadIdx.x] = a;
        __syncthreads();
        for (int w = kRedThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out6[k] = sh[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- adjoint
// Seeds lam = dL/dM of the objectives: kinetic energy
// L = 1/2 sum_fluid rho |u|^2, or the wall shear force (linear in Pi: the
// weight of Pi_xy / Pi_xz at the wall-adjacent layers, zero elsewhere).
__global__ void adjoint_seed_kernel(const float* __restrict__ st, float* __restrict__ lam, StepParams p,
                                    int objective) {
    const Geometry& g = p.geo;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.n[0]);
    const int y = (int)((n / g.n[0]) % g.n[1]);
    const int z = (int)(n / ((long long)g.n[0] * g.n[1]));
    const bool fl = is_fluid(g, x, y, z);
    if (objective == 1) {
#pragma unroll
        for (int k = 0; k < 10; ++k) lam[k * g.N + n] = 0.0f;
        if (fl) {
            lam[7 * g.N + n] = (float)wall_shear_weight(g, p, y, z, 1);
            lam[8 * g.N + n] = (float)wall_shear_weight(g, p, y, z, 2);
        }
        return;
    }
    const float rho = 1.0f + st[n];
    const float ux = st[g.N + n], uy = st[2 * g.N + n], uz = st[3 * g.N + n];
    lam[n] = fl ? 0.5f * (ux * ux + uy * uy + uz * uz) : 0.0f;
    lam[g.N + n] = fl ? rho * ux : 0.0f;
    lam[2 * g.N + n] = fl ? rho * uy : 0.0f;
    lam[3 * g.N + n] = fl ? rho * uz : 0.0f;
#pragma unroll
    for (int k = 4; k < 10; ++k) lam[k * g.N + n] = 0.0f;
}

// Sensitivity of the arriving population along c to the new moments at
// its node: dM'/df for M' = (rho', u', Pi'), with rho' = sum f,
// u' = sum f c / rho', Pi' = sum f c c - rho' u' u' - rho'/3 delta:
//   d rho'/df = 1, d u'/df = (c - u') / rho',
//   d Pi'_ab/df = (c_a - u'_a)(c_b - u'_b) - delta_ab / 3.
template <int I>
__device__ __forceinline__ float arrival_adjoint(const float lam[10], float rho1, const float u1[3]) {
    constexpr int X = cx_of(I), Y = cy_of(I), Z = cz_of(I);
    const float dx = X - u1[0], dy = Y - u1[1], dz = Z - u1[2];
    const float third = 1.0f / 3.0f;
    float s = lam[0] + (lam[1] * dx + lam[2] * dy + lam[3] * dz) / rho1;
    s += lam[4] * (dx * dx - third) + lam[5] * (dy * dy - third) + lam[6] * (dz * dz - third);
    s += lam[7] * dx * dy + lam[8] * dx * dz + lam[9] * dy * dz;
    return s;
}

// lf * d(w P(c_I))/d(drho, u, Pi, g) added into acc[13] (see the form of P
// in tslb_device.h; Pi off-diagonals are single stored variables).
template <int I>
__device__ __forceinline__ void emit_adjoint(const NodeTerms& t, float omo, float lf, float acc[13]) {
    constexpr int X = cx_of(I), Y = cy_of(I), Z = cz_of(I);
    constexpr float W = w216_of(I) * kInv216;
    const float c[3] = {(float)X, (float)Y, (float)Z};
    const float cu = X * t.u[0] + Y * t.u[1] + Z * t.u[2];
    const float cpc = X * X * t.p[0] + Y * Y * t.p[1] + Z * Z * t.p[2] +
                      2.0f * (X * Y * t.p[3] + X * Z * t.p[4] + Y * Z * t.p[5]);
    const float cg = X * t.rg[0] + Y * t.rg[1] + Z * t.rg[2];
    const float wl = W * lf;
    const float E = cu * (3.0f + 4.5f * cu) - 1.5f * t.u2 + 4.5f * cu * (cu * cu - t.u2);
    // d/d drho: 1 + E + 3 c.g  (rho = 1 + drho multiplies E and the force term)
    acc[0] += wl * (1.0f + E + 3.0f * cg / t.rho);
    // d/du_a
    const float pc[3] = {X * t.p[0] + Y * t.p[3] + Z * t.p[4], X * t.p[3] + Y * t.p[1] + Z * t.p[5],
                         X * t.p[4] + Y * t.p[5] + Z * t.p[2]};
    const float ca = 3.0f + 9.0f * cu + 13.5f * cu * cu - 4.5f * t.u2;
    const float ua = 3.0f + 9.0f * cu;
    const float na = 13.5f * cpc - 4.5f * t.trp;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        acc[1 + a] += wl * (t.rho * (c[a] * ca - t.u[a] * ua) + omo * (c[a] * na - 9.0f * pc[a]));
    // d/dPi_aa
#pragma unroll
    for (int a = 0; a < 3; ++a)
        acc[4 + a] += wl * omo * (c[a] * c[a] * (4.5f + 13.5f * cu) - 1.5f - 4.5f * cu - 9.0f * c[a] * t.u[a]);
    // d/dPi_ab, a < b: (xy, xz, yz)
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a = pa[k], b = pb[k];
        acc[7 + k] += wl * omo * (c[a] * c[b] * (9.0f + 27.0f * cu) - 9.0f * (c[a] * t.u[b] + c[b] * t.u[a]));
    }
    // d/dg_a: 3 rho c_a
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[10 + a] += wl * 3.0f * t.rho * c[a];
}

// Reverse of one step at node y: every population y emitted went to the
// downstream node y + c_i (or back to y itself when the upstream node of
// y along c_i is solid); its sensitivity is gathered there and pulled back
// through the Jacobian of the emission.  A gather, race free like the
// forward update.
__global__ void __launch_bounds__(256) adjoint_step_kernel(const float* __restrict__ st0,
                                                           const float* __restrict__ st1,
                                                           const float* __restrict__ lam1,
                                                           float* __restrict__ lam0, float* __restrict__ dg,
                                                           StepParams p) {
    const Geometry& g = p.geo;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.n[0]);
    const int y = (int)((n / g.n[0]) % g.n[1]);
    const int z = (int)(n / ((long long)g.n[0] * g.n[1]));
    // walls emit nothing; fluid and ghost nodes emit (a ghost node is an
    // ordinary source of the update, Section 2.3)
    if (is_solid(g, x, y, z)) {
#pragma unroll
        for (int k = 0; k < 10; ++k) lam0[k * g.N + n] = 0.0f;
        return;
    }
    const bool fluid = is_fluid(g, x, y, z);
    float m[10], gg[3];
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = st0[k * g.N + n];
#pragma unroll
    for (int a = 0; a < 3; ++a) gg[a] = p.gfield ? p.gfield[a * g.N + n] : p.force[a];
    const NodeTerms t = node_terms(m, gg);
    const float omo = omo_at(p, z);
    float acc[13];
#pragma unroll
    for (int k = 0; k < 13; ++k) acc[k] = 0.0f;
    Unroll<0, 27>::run([&]<int I>() {
        constexpr int X = cx_of(I), Y = cy_of(I), Z = cz_of(I);
        // downstream node y + c_I receives this node's population I
        int dx = x + X, dy = y + Y, dz = z + Z;
        if ((g.periodic >> 0) & 1) dx = dx < 0 ? dx + g.n[0] : (dx >= g.n[0] ? dx - g.n[0] : dx);
        if ((g.periodic >> 1) & 1) dy = dy < 0 ? dy + g.n[1] : (dy >= g.n[1] ? dy - g.n[1] : dy);
        if ((g.periodic >> 2) & 1) dz = dz < 0 ? dz + g.n[2] : (dz >= g.n[2] ? dz - g.n[2] : dz);
        const bool inside = dx >= 0 && dx < g.n[0] && dy >= 0 && dy < g.n[1] && dz >= 0 && dz < g.n[2];
        if (inside && is_fluid(g, dx, dy, dz)) {
            const long long d = dx + (long long)g.n[0] * (dy + (long long)g.n[1] * dz);
            float l[10], u1[3];
#pragma unroll
            for (int k = 0; k < 10; ++k) l[k] = lam1[k * g.N + d];
            const float rho1 = 1.0f + st1[d];
#pragma unroll
            for (int a = 0; a < 3; ++a) u1[a] = st1[(1 + a) * g.N + d];
            emit_adjoint<I>(t, omo, arrival_adjoint<I>(l, rho1, u1), acc);
        }
        // upstream node y - c_I solid: y's own population 26 - I came back as I
        int ux = x - X, uy = y - Y, uz = z - Z;
        if ((g.periodic >> 0) & 1) ux = ux < 0 ? ux + g.n[0] : (ux >= g.n[0] ? ux - g.n[0] : ux);
        if ((g.periodic >> 1) & 1) uy = uy < 0 ? uy + g.n[1] : (uy >= g.n[1] ? uy - g.n[1] : uy);
        if ((g.periodic >> 2) & 1) uz = uz < 0 ? uz + g.n[2] : (uz >= g.n[2] ? uz - g.n[2] : uz);
        if (fluid && is_solid(g, ux, uy, uz)) {
            float l[10], u1[3];
#pragma unroll
            for (int k = 0; k < 10; ++k) l[k] = lam1[k * g.N + n];
            const float rho1 = 1.0f + st1[n];
#pragma unroll
            for (int a = 0; a < 3; ++a) u1[a] = st1[(1 + a) * g.N + n];
            emit_adjoint<26 - I>(t, omo, arrival_adjoint<I>(l, rho1, u1), acc);
        }
    });
#pragma unroll
    for (int k = 0; k < 10; ++k) lam0[k * g.N + n] = acc[k];
    if (dg)
#pragma unroll
        for (int a = 0; a < 3; ++a) dg[a * g.N + n] += acc[10 + a];
}

// The transpose of the ghost refill, in place on a sensitivity field lam
// (10 N floats): every ghost node copied the ten moments of its interior
// neighbour (rho and Pi^neq only on an inlet disc, whose velocity is imposed
// and does not depend on the state), so its sensitivities are added to that
// neighbour's and cleared.  Threads enumerate the interior layers next to
// the ghost faces (a node on several of them is done once, by the first);
// each gathers, in a fixed order, from the ghost nodes among its 26
// neighbours that copy it.  Every ghost copies exactly one node, so the
// update in place is race free.
__global__ void ghost_fold_kernel(float* __restrict__ lam, StepParams p, InletParams q, long long off1,
                                  long long off2, long long off3, long long off4, long long off5, long long total) {
    const Geometry& g = p.geo;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= total) return;
    const long long offs[6] = {0, off1, off2, off3, off4, off5};
    int f = 5;
    while (f > 0 && tid < offs[f]) --f;
    if (q.face_kind[f] != kInlet && q.face_kind[f] != kOutlet) return;
    const int d = f >> 1;
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    const long long local = tid - offs[f];
    auto inner = [&](int face) { return (face & 1) ? g.n[face >> 1] - 2 : 1; };
    int c[3];
    c[d] = inner(f);
    c[d1] = (int)(local % g.n[d1]);
    c[d2] = (int)(local / g.n[d1]);
    if (c[d2] >= g.n[d2]) return;
    if (!is_fluid(g, c[0], c[1], c[2])) return;
    for (int f2 = 0; f2 < f; ++f2)
        if ((q.face_kind[f2] == kInlet || q.face_kind[f2] == kOutlet) && c[f2 >> 1] == inner(f2)) return;
    const long long n = c[0] + (long long)g.n[0] * (c[1] + (long long)g.n[1] * c[2]);
    float acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = lam[k * g.N + n];
    for (int o = 0; o < 27; ++o) {
        const int e[3] = {c[0] + o % 3 - 1, c[1] + (o / 3) % 3 - 1, c[2] + o / 9 - 1};
        if (o == 13 || e[0] < 0 || e[0] >= g.n[0] || e[1] < 0 || e[1] >= g.n[1] || e[2] < 0 || e[2] >= g.n[2])
            continue;
        bool ghost = false, src = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int cf = e[a];
            if (e[a] == 0 && ((g.lo_ghost >> a) & 1)) {
                ghost = true;
                cf = 1;
            }
            if (e[a] == g.n[a] - 1 && ((g.hi_ghost >> a) & 1)) {
                ghost = true;
                cf = g.n[a] - 2;
            }
            src &= cf == c[a];
        }
        if (!ghost || !src || is_solid(g, e[0], e[1], e[2])) continue;
        const long long m = e[0] + (long long)g.n[0] * (e[1] + (long long)g.n[1] * e[2]);
        float u[3];
        const bool imposed = inlet_velocity(g, q, p.dims, 0, m, e, u);
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            if (!(imposed && k >= 1 && k <= 3)) acc[k] += lam[k * g.N + m];
            lam[k * g.N + m] = 0.0f;
        }
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) lam[k * g.N + n] = acc[k];
}

template <class S>
hipError_t ghost_fill_t(void* st, const StepParams& p, const InletParams& q, int64_t t, int x_done, hipStream_t s) {
    long long area[6];
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
        area[f] = (q.face_kind[f] == kInlet || q.face_kind[f] == kOutlet) ? (long long)p.geo.n[d1] * p.geo.n[d2] : 0;
    }
    long long off[7] = {0};
    for (int f = 0; f < 6; ++f) off[f + 1] = off[f] + area[f];
    if (off[6] == 0) return hipSuccess;
    const int block = 256;
    const long long grid = (off[6] + block - 1) / block;
    hipLaunchKernelGGL(ghost_fill_kernel<S>, dim3((unsigned)grid), dim3(block), 0, s, (typename S::T*)st, p, q, t,
                       off[1], off[2], off[3], off[4], off[5], off[6], x_done);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ghost_fill(int storage, void* st, const StepParams& p, const InletParams& q, int64_t t,
                             int x_done, hipStream_t s) {
    switch (storage) {
    case 0: return ghost_fill_t<StoreF32>(st, p, q, t, x_done, s);
    case 1: return ghost_fill_t<StoreF16>(st, p, q, t, x_done, s);
    case 2: return ghost_fill_t<StoreBF16>(st, p, q, t, x_done, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pack(int storage, const float* rho, const float* u, const float* pi, int rho_dev, void* st,
                       const StepParams& p, hipStream_t s) {
    const int block = 256;
    const unsigned grid = (unsigned)((p.geo.N + block - 1) / block);
    switch (storage) {
    case 0: hipLaunchKernelGGL(pack_kernel<StoreF32>, dim3(grid), dim3(block), 0, s, rho, u, pi, rho_dev, (float*)st, p); break;
    case 1: hipLaunchKernelGGL(pack_kernel<StoreF16>, dim3(grid), dim3(block), 0, s, rho, u, pi, rho_dev, (__half*)st, p); break;
    case 2: hipLaunchKernelGGL(pack_kernel<StoreBF16>, dim3(grid), dim3(block), 0, s, rho, u, pi, rho_dev, (uint16_t*)st, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpack(int storage, const void* st, float* rho, float* u, float* pi, int rho_dev,
                         const StepParams& p, hipStream_t s) {
    const int block = 256;
    const unsigned grid = (unsigned)((p.geo.N + block - 1) / block);
    switch (storage) {
    case 0: hipLaunchKernelGGL(unpack_kernel<StoreF32>, dim3(grid), dim3(block), 0, s, (const float*)st, rho, u, pi, rho_dev, p); break;
    case 1: hipLaunchKernelGGL(unpack_kernel<StoreF16>, dim3(grid), dim3(block), 0, s, (const __half*)st, rho, u, pi, rho_dev, p); break;
    case 2: hipLaunchKernelGGL(unpack_kernel<StoreBF16>, dim3(grid), dim3(block), 0, s, (const uint16_t*)st, rho, u, pi, rho_dev, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ghost_fold(float* lam, const StepParams& p, const InletParams& q, hipStream_t s) {
    long long area[6];
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
        area[f] = (q.face_kind[f] == kInlet || q.face_kind[f] == kOutlet) ? (long long)p.geo.n[d1] * p.geo.n[d2] : 0;
    }
    long long off[7] = {0};
    for (int f = 0; f < 6; ++f) off[f + 1] = off[f] + area[f];
    if (off[6] == 0) return hipSuccess;
    const int block = 256;
    const long long grid = (off[6] + block - 1) / block;
    hipLaunchKernelGGL(ghost_fold_kernel, dim3((unsigned)grid), dim3(block), 0, s, lam, p, q, off[1], off[2], off[3],
                       off[4], off[5], off[6]);
    return hipGetLastError();
}

hipError_t launch_reduce(int storage, const void* st, double* partials, int nblocks, double* out6,
                         const StepParams& p, hipStream_t s) {
    switch (storage) {
    case 0: hipLaunchKernelGGL(reduce_partial_kernel<StoreF32>, dim3(nblocks), dim3(kRedThreads), 0, s, (const float*)st, partials, p); break;
    case 1: hipLaunchKernelGGL(reduce_partial_kernel<StoreF16>, dim3(nblocks), dim3(kRedThreads), 0, s, (const __half*)st, partials, p); break;
    case 2: hipLaunchKernelGGL(reduce_partial_kernel<StoreBF16>, dim3(nblocks), dim3(kRedThreads), 0, s, (const uint16_t*)st, partials, p); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, nblocks, out6);
    return hipGetLastError();
}

// ---------------------------------------------------------------- copy
// Plain device-to-device stream of 16-byte words: every word read once and
// written once, each block moving 4 x 256 consecutive words (four loads in
// flight per thread), non-temporal loads and stores (nothing is re-read, so
// nothing is worth keeping in the caches).  The fastest of the plain copies
// measured on MI355X; its rate is the practical read+write bandwidth ceiling
// the update's own rate is compared with.
__global__ void __launch_bounds__(256) stream_copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                          long long n4) {
    const long long base = (long long)blockIdx.x * 1024 + threadIdx.x;
    float4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long i = base + 256 * k;
        if (i < n4) {
            const float* p = reinterpret_cast<const float*>(src + i);
            v[k] = make_float4(__builtin_nontemporal_load(p), __builtin_nontemporal_load(p + 1),
                               __builtin_nontemporal_load(p + 2), __builtin_nontemporal_load(p + 3));
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long i = base + 256 * k;
        if (i < n4) {
            float* p = reinterpret_cast<float*>(dst + i);
            __builtin_nontemporal_store(v[k].x, p);
            __builtin_nontemporal_store(v[k].y, p + 1);
            __builtin_nontemporal_store(v[k].z, p + 2);
            __builtin_nontemporal_store(v[k].w, p + 3);
        }
    }
}

hipError_t launch_stream_copy(const void* src, void* dst, long long n4, hipStream_t s) {
    if (n4 <= 0) return hipSuccess;
    const long long blocks = (n4 + 1023) / 1024;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (const float4*)src, (float4*)dst, n4);
    return hipGetLastError();
}

hipError_t launch_adjoint_seed(const float* st, float* lam, const StepParams& p, int objective, hipStream_t s) {
    const int block = 256;
    const unsigned grid = (unsigned)((p.geo.N + block - 1) / block);
    hipLaunchKernelGGL(adjoint_seed_kernel, dim3(grid), dim3(block), 0, s, st, lam, p, objective);
    return hipGetLastError();
}

hipError_t launch_adjoint_step(const float* st0, const float* st1, const float* lam1, float* lam0, float* dg,
                               const StepParams& p, hipStream_t s) {
    const int block = 256;
    const unsigned grid = (unsigned)((p.geo.N + block - 1) / block);
    hipLaunchKernelGGL(adjoint_step_kernel, dim3(grid), dim3(block), 0, s, st0, st1, lam1, lam0, dg, p);
    return hipGetLastError();
}

}  // namespace tslb
