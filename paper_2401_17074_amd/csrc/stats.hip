// On-device velocity statistics of the turbulence benchmarks (Section 3.1:
// mean profile, second- and third-order moments over the homogeneous
// directions and time; Section 3.2: centreline velocity and half-width of
// the jet from the time-averaged field).  Sums are FP64.
//
//   profile : for every index j along the profile axis, the sums over the
//             fluid nodes of plane j of 1, u_a, u_a u_b, u_a^3 (13 values),
//             accumulated over samples.  A sample is two launches: per-block
//             partials in a fixed order, then one thread per (plane, value)
//             adds them up in a fixed order (deterministic).
//   field   : per-node sums of u_a and u_a u_b (9 FP64 arrays).
//   jet     : one block per cross-section bins the mean axial velocity by
//             k = floor(r) in LDS, then finds U_c and r_1/2.
#include "tslb_internal.h"

namespace tslb {
namespace {

constexpr int kStatBlock = 256;

// node index of in-plane position k of plane j along axis
__device__ __forceinline__ long long plane_node(const Geometry& g, int axis, int j, long long k, int c[3]) {
    const int d1 = axis == 0 ? 1 : 0, d2 = axis == 2 ? 1 : 2;
    c[axis] = j;
    c[d1] = (int)(k % g.n[d1]);
    c[d2] = (int)(k / g.n[d1]);
    return c[0] + (long long)g.n[0] * (c[1] + (long long)g.n[1] * c[2]);
}

template <class S>
__global__ void __launch_bounds__(kStatBlock) profile_partial_kernel(const typename S::T* __restrict__ st,
                                                                     double* __restrict__ part, StepParams p,
                                                                     int axis, int blocks_per_plane) {
    const Geometry& g = p.geo;
    const int j = blockIdx.y;
    const int d1 = axis == 0 ? 1 : 0, d2 = axis == 2 ? 1 : 2;
    const long long plane = (long long)g.n[d1] * g.n[d2];
    double acc[13];
#pragma unroll
    for (int q = 0; q < 13; ++q) acc[q] = 0.0;
    for (long long k = (long long)blockIdx.x * kStatBlock + threadIdx.x; k < plane;
         k += (long long)blocks_per_plane * kStatBlock) {
        int c[3];
        const long long n = plane_node(g, axis, j, k, c);
        if (!is_fluid(g, c[0], c[1], c[2])) continue;
        const double u0 = S::load(st[1 * g.N + n], p.inv_scale[1]);
        const double u1 = S::load(st[2 * g.N + n], p.inv_scale[1]);
        const double u2 = S::load(st[3 * g.N + n], p.inv_scale[1]);
        acc[0] += 1.0;
        acc[1] += u0;
        acc[2] += u1;
        acc[3] += u2;
        acc[4] += u0 * u0;
        acc[5] += u1 * u1;
        acc[6] += u2 * u2;
        acc[7] += u0 * u1;
        acc[8] += u0 * u2;
        acc[9] += u1 * u2;
        acc[10] += u0 * u0 * u0;
        acc[11] += u1 * u1 * u1;
        acc[12] += u2 * u2 * u2;
    }
    // block reduction in a fixed order
    __shared__ double red[13][kStatBlock];
#pragma unroll
    for (int q = 0; q < 13; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = kStatBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < 13; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 13)
        part[((long long)j * blocks_per_plane + blockIdx.x) * 13 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void profile_final_kernel(const double* __restrict__ part, double* __restrict__ sums, int n_axis,
                                     int blocks_per_plane) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_axis * 13) return;
    const int j = i / 13, q = i % 13;
    double s = 0.0;
    for (int b = 0; b < blocks_per_plane; ++b) s += part[((long long)j * blocks_per_plane + b) * 13 + q];
    sums[i] += s;
}

template <class S>
__global__ void __launch_bounds__(kStatBlock) field_sample_kernel(const typename S::T* __restrict__ st,
                                                                  double* __restrict__ s, StepParams p) {
    const long long N = p.geo.N;
    const long long n = (long long)blockIdx.x * kStatBlock + threadIdx.x;
    if (n >= N) return;
    const double u0 = S::load(st[1 * N + n], p.inv_scale[1]);
    const double u1 = S::load(st[2 * N + n], p.inv_scale[1]);
    const double u2 = S::load(st[3 * N + n], p.inv_scale[1]);
    s[0 * N + n] += u0;
    s[1 * N + n] += u1;
    s[2 * N + n] += u2;
    s[3 * N + n] += u0 * u0;
    s[4 * N + n] += u1 * u1;
    s[5 * N + n] += u2 * u2;
    s[6 * N + n] += u0 * u1;
    s[7 * N + n] += u0 * u2;
    s[8 * N + n] += u1 * u2;
}

__global__ void __launch_bounds__(kStatBlock) field_moments_kernel(const double* __restrict__ s, long long N,
                                                                   double inv_ns, float* __restrict__ mean,
                                                                   float* __restrict__ cov) {
    const long long n = (long long)blockIdx.x * kStatBlock + threadIdx.x;
    if (n >= N) return;
    double m[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) m[a] = s[a * N + n] * inv_ns;
    if (mean) {
#pragma unroll
        for (int a = 0; a < 3; ++a) mean[a * N + n] = (float)m[a];
    }
    if (cov) {
        const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int k = 0; k < 6; ++k) cov[k * N + n] = (float)(s[(3 + k) * N + n] * inv_ns - m[A[k]] * m[B[k]]);
    }
}

constexpr int kJetBlock = 256;

// One block per cross-section j along `axis`.  Bin k = floor(r) holds the
// count, the summed radius and the summed mean axial velocity of its nodes.
// Each bin is owned by one thread, which visits the nodes of its annulus
// k <= r < k + 1 row by row and, within a row, in increasing coordinate
// (a fixed order, so the sums do not depend on scheduling); thread 0 then
// walks the bins.
__global__ void __launch_bounds__(kJetBlock) jet_axis_kernel(const double* __restrict__ s, Geometry g, int axis,
                                                             float c1, float c2, double inv_ns, int nbins,
                                                             float* __restrict__ uc, float* __restrict__ rhalf) {
    extern __shared__ double bins[];  // 3 * nbins: count, sum r, sum u
    const int j = blockIdx.x;
    const int d1 = axis == 0 ? 1 : 0, d2 = axis == 2 ? 1 : 2;
    const int n1 = g.n[d1], n2 = g.n[d2];
    const double* __restrict__ ua = s + (long long)axis * g.N;
    for (int b = threadIdx.x; b < nbins; b += kJetBlock) {
        double cnt = 0.0, sr = 0.0, su = 0.0;
        const double bo = (double)b + 1.0, bi = (double)b;
        const int y0 = max(0, (int)floor((double)c2 - bo) - 1), y1 = min(n2 - 1, (int)ceil((double)c2 + bo) + 1);
        for (int y = y0; y <= y1; ++y) {
            const double r2 = (double)y - (double)c2;
            const double qo = bo * bo - r2 * r2;
            if (qo <= 0.0) continue;  // every node of this row has r >= b + 1
            const double qi = bi * bi - r2 * r2;
            const double so = sqrt(qo), si = qi > 0.0 ? sqrt(qi) : 0.0;
            // the annulus meets the row in [c1 - so, c1 - si] and [c1 + si, c1 + so];
            // both ranges are widened by one node and every candidate is tested
            const int xl0 = max(0, (int)floor((double)c1 - so) - 1);
            const int xl1 = min(n1 - 1, (int)ceil((double)c1 - si) + 1);
            int xr0 = max(0, (int)floor((double)c1 + si) - 1);
            const int xr1 = min(n1 - 1, (int)ceil((double)c1 + so) + 1);
            if (xr0 <= xl1) xr0 = xl1 + 1;
            for (int pass = 0; pass < 2; ++pass) {
                const int xa = pass == 0 ? xl0 : xr0, xb = pass == 0 ? xl1 : xr1;
                for (int x = xa; x <= xb; ++x) {
                    const double r1 = (double)x - (double)c1;
                    const double r = sqrt(r1 * r1 + r2 * r2);
                    if ((int)floor(r) != b) continue;
                    int c[3];
                    c[axis] = j;
                    c[d1] = x;
                    c[d2] = y;
                    const long long n = c[0] + (long long)g.n[0] * (c[1] + (long long)g.n[1] * c[2]);
                    cnt += 1.0;
                    sr += r;
                    su += ua[n] * inv_ns;
                }
            }
        }
        bins[b] = cnt;
        bins[nbins + b] = sr;
        bins[2 * nbins + b] = su;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double u0 = bins[2 * nbins] / bins[0];
    const double half = 0.5 * u0;
    double rh = -1.0;
    int prev = 0;
    for (int b = 1; b < nbins; ++b) {
        if (bins[b] == 0.0) continue;
        const double pb = bins[2 * nbins + b] / bins[b];
        if (pb <= half) {
            const double pp = bins[2 * nbins + prev] / bins[prev];
            const double rp = bins[nbins + prev] / bins[prev], rb = bins[nbins + b] / bins[b];
            rh = rp + (rb - rp) * (pp - half) / (pp - pb);
            break;
        }
        prev = b;
    }
    uc[j] = (float)u0;
    rhalf[j] = (float)rh;
}

template <class S>
hipError_t profile_s(const void* st, double* part, double* sums, const StepParams& p, int axis, int bpp,
                     hipStream_t s) {
    const int n_axis = p.geo.n[axis];
    hipLaunchKernelGGL(profile_partial_kernel<S>, dim3(bpp, n_axis), dim3(kStatBlock), 0, s,
                       (const typename S::T*)st, part, p, axis, bpp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int total = n_axis * 13;
    hipLaunchKernelGGL(profile_final_kernel, dim3((total + 255) / 256), dim3(256), 0, s, part, sums, n_axis, bpp);
    return hipGetLastError();
}

template <class S>
hipError_t field_s(const void* st, double* fs, const StepParams& p, hipStream_t s) {
    const unsigned grid = (unsigned)((p.geo.N + kStatBlock - 1) / kStatBlock);
    hipLaunchKernelGGL(field_sample_kernel<S>, dim3(grid), dim3(kStatBlock), 0, s, (const typename S::T*)st, fs, p);
    return hipGetLastError();
}

}  // namespace

int stats_blocks_per_plane(const Geometry& g, int axis) {
    const int d1 = axis == 0 ? 1 : 0, d2 = axis == 2 ? 1 : 2;
    const long long plane = (long long)g.n[d1] * g.n[d2];
    long long b = (plane + 4 * kStatBlock - 1) / (4 * kStatBlock);
    return (int)(b < 1 ? 1 : (b > 64 ? 64 : b));
}

hipError_t launch_stats_profile(int storage, const void* st, double* part, double* sums, const StepParams& p,
                                int axis, hipStream_t s) {
    const int bpp = stats_blocks_per_plane(p.geo, axis);
    switch (storage) {
    case 0: return profile_s<StoreF32>(st, part, sums, p, axis, bpp, s);
    case 1: return profile_s<StoreF16>(st, part, sums, p, axis, bpp, s);
    case 2: return profile_s<StoreBF16>(st, part, sums, p, axis, bpp, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_stats_field(int storage, const void* st, double* fs, const StepParams& p, hipStream_t s) {
    switch (storage) {
    case 0: return field_s<StoreF32>(st, fs, p, s);
    case 1: return field_s<StoreF16>(st, fs, p, s);
    case 2: return field_s<StoreBF16>(st, fs, p, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_stats_field_moments(const double* fs, long long N, double inv_ns, float* mean, float* cov,
                                      hipStream_t s) {
    const unsigned grid = (unsigned)((N + kStatBlock - 1) / kStatBlock);
    hipLaunchKernelGGL(field_moments_kernel, dim3(grid), dim3(kStatBlock), 0, s, fs, N, inv_ns, mean, cov);
    return hipGetLastError();
}

int stats_jet_bins(const Geometry& g, int axis, float c1, float c2) {
    const int d1 = axis == 0 ? 1 : 0, d2 = axis == 2 ? 1 : 2;
    double rmax = 0.0;
    const double cx[2] = {0.0, (double)(g.n[d1] - 1)}, cy[2] = {0.0, (double)(g.n[d2] - 1)};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const double r1 = cx[a] - c1, r2 = cy[b] - c2;
            const double r = sqrt(r1 * r1 + r2 * r2);
            if (r > rmax) rmax = r;
        }
    return (int)floor(rmax) + 1;
}

hipError_t launch_stats_jet(const double* fs, const Geometry& g, int axis, float c1, float c2, double inv_ns,
                            float* uc, float* rhalf, hipStream_t s) {
    const int nbins = stats_jet_bins(g, axis, c1, c2);
    const size_t lds = sizeof(double) * 3 * (size_t)nbins;
    hipLaunchKernelGGL(jet_axis_kernel, dim3(g.n[axis]), dim3(kJetBlock), lds, s, fs, g, axis, c1, c2, inv_ns, nbins,
                       uc, rhalf);
    return hipGetLastError();
}

}  // namespace tslb
