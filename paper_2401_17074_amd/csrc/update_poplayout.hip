// Population-layout variant of the update: the storage scheme of the paper's
// own GPU code (Section 2.2, the remark on memory footprint), i.e. one set of
// 27 populations kept next to the ten moment arrays.  A step is two passes:
//
//   push    every non-solid node rebuilds its 27 post-collision populations
//           from its own level-t moments and writes each into the slot of the
//           node it streams to, x + c_i.  A population aimed at a solid node
//           is written into the emitter's own slot of the opposite direction
//           (half-way bounce-back).  Every slot read by a fluid node has
//           exactly one writer, so a single population set needs no A/B copy.
//   moments every fluid node sums its 27 arrived populations and stores the
//           level-(t+1) moments.
//
// Populations are kept as FP32 scaled deviations G = 216 w P, the values the
// fused kernels exchange through LDS, so both forms compute the same update.
// Per node and step the passes move 10 + 27 + 27 + 10 values: against the
// 10 + 10 of the moment-only form this is the layout ablation.
#include "tslb_internal.h"

namespace tslb {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int wrap_axis(int v, int n, bool periodic) {
    if (periodic) v = v < 0 ? v + n : (v >= n ? v - n : v);
    return v;
}

template <class S, int ORDER, bool FIELD>
__global__ void __launch_bounds__(kBlock) push_kernel(const typename S::T* __restrict__ in, float* __restrict__ pop,
                                                      StepParams p) {
    const Geometry& g = p.geo;
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.n[0]);
    const int y = (int)((n / g.n[0]) % g.n[1]);
    const int z = (int)(n / ((long long)g.n[0] * g.n[1]));
    if (is_solid(g, x, y, z)) return;

    float m[10], gg[3];
    m[0] = S::load(in[n], p.inv_scale[0]);
#pragma unroll
    for (int q = 1; q < 4; ++q) m[q] = S::load(in[q * g.N + n], p.inv_scale[1]);
#pragma unroll
    for (int q = 4; q < 10; ++q) m[q] = S::load(in[q * g.N + n], p.inv_scale[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) gg[a] = FIELD ? p.gfield[a * g.N + n] : p.force[a];
    const NodeTerms t = node_terms(m, gg);
    const float omo = omo_at(p, z);

    Unroll<0, 27>::run([&]<int I>() {
        constexpr int X = cx_of(I), Y = cy_of(I), Z = cz_of(I);
        const int tx = wrap_axis(x + X, g.n[0], g.periodic & 1);
        const int ty = wrap_axis(y + Y, g.n[1], (g.periodic >> 1) & 1);
        const int tz = wrap_axis(z + Z, g.n[2], (g.periodic >> 2) & 1);
        // leaving the array happens only to ghost nodes on an open face
        if (tx < 0 || tx >= g.n[0] || ty < 0 || ty >= g.n[1] || tz < 0 || tz >= g.n[2]) return;
        const float G = emit_dev<I, ORDER>(t, omo);
        if (is_solid(g, tx, ty, tz))
            pop[(26 - I) * g.N + n] = G;
        else
            pop[I * g.N + tx + (long long)g.n[0] * (ty + (long long)g.n[1] * tz)] = G;
    });
}

template <class S>
__global__ void __launch_bounds__(kBlock) moments_kernel(const float* __restrict__ pop, typename S::T* __restrict__ out,
                                                         StepParams p) {
    const Geometry& g = p.geo;
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.n[0]);
    const int y = (int)((n / g.n[0]) % g.n[1]);
    const int z = (int)(n / ((long long)g.n[0] * g.n[1]));
    if (!is_fluid(g, x, y, z)) return;
    MomentSums a;
    a.zero();
    Unroll<0, 27>::run([&]<int I>() { a.template add<I>(pop[I * g.N + n]); });
    float m[10];
    finalize(a, m);
    out[n] = S::store(m[0], p.scale[0]);
#pragma unroll
    for (int q = 1; q < 4; ++q) out[q * g.N + n] = S::store(m[q], p.scale[1]);
#pragma unroll
    for (int q = 4; q < 10; ++q) out[q * g.N + n] = S::store(m[q], p.scale[2]);
}

template <class S, int ORDER>
hipError_t launch_o(const void* in, void* out, float* pop, const StepParams& p, hipStream_t s) {
    const unsigned grid = (unsigned)((p.geo.N + kBlock - 1) / kBlock);
    const auto* src = (const typename S::T*)in;
    if (p.gfield)
        hipLaunchKernelGGL((push_kernel<S, ORDER, true>), dim3(grid), dim3(kBlock), 0, s, src, pop, p);
    else
        hipLaunchKernelGGL((push_kernel<S, ORDER, false>), dim3(grid), dim3(kBlock), 0, s, src, pop, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(moments_kernel<S>, dim3(grid), dim3(kBlock), 0, s, pop, (typename S::T*)out, p);
    return hipGetLastError();
}

template <class S>
hipError_t launch_s(const void* in, void* out, float* pop, const StepParams& p, hipStream_t s) {
    return p.order == 2 ? launch_o<S, 2>(in, out, pop, p, s) : launch_o<S, 3>(in, out, pop, p, s);
}

}  // namespace

hipError_t launch_update_poplayout(int storage, const void* in, void* out, float* pop, const StepParams& p,
                                   hipStream_t s) {
    if (p.geo.N * 27 >= (1LL << 62) || (p.geo.N + kBlock - 1) / kBlock >= (1LL << 31)) return hipErrorInvalidValue;
    switch (storage) {
    case 0: return launch_s<StoreF32>(in, out, pop, p, s);
    case 1: return launch_s<StoreF16>(in, out, pop, p, s);
    case 2: return launch_s<StoreBF16>(in, out, pop, p, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace tslb
