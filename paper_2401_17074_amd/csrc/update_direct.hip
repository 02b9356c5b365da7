// Direct update kernel: one thread per node, 27 upstream moment sets read
// straight from global memory (the caches absorb the reuse).  It is the
// plainest form of the pull update of Section 2.2 and serves as the
// cross-check of the tiled kernel.
#include "tslb_internal.h"

namespace tslb {
namespace {

template <class S>
__device__ __forceinline__ void load_moments(const typename S::T* st, long long N, long long n,
                                             const float inv[3], float m[10]) {
    m[0] = S::load(st[n], inv[0]);
#pragma unroll
    for (int q = 1; q < 4; ++q) m[q] = S::load(st[q * N + n], inv[1]);
#pragma unroll
    for (int q = 4; q < 10; ++q) m[q] = S::load(st[q * N + n], inv[2]);
}

template <class S, int ORDER>
__global__ void __launch_bounds__(256) update_direct_kernel(const typename S::T* __restrict__ in,
                                                            typename S::T* __restrict__ out, StepParams p) {
    const Geometry& g = p.geo;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.n[0]);
    const int y = (int)((n / g.n[0]) % g.n[1]);
    const int z = (int)(n / ((long long)g.n[0] * g.n[1]));
    if (!is_fluid(g, x, y, z)) return;

    MomentSums acc;
    acc.zero();
    Unroll<0, 27>::run([&]<int I>() {
        constexpr int X = cx_of(I), Y = cy_of(I), Z = cz_of(I);
        int sx = x - X, sy = y - Y, sz = z - Z;
        if ((g.periodic >> 0) & 1) sx = sx < 0 ? sx + g.n[0] : (sx >= g.n[0] ? sx - g.n[0] : sx);
        if ((g.periodic >> 1) & 1) sy = sy < 0 ? sy + g.n[1] : (sy >= g.n[1] ? sy - g.n[1] : sy);
        if ((g.periodic >> 2) & 1) sz = sz < 0 ? sz + g.n[2] : (sz >= g.n[2] ? sz - g.n[2] : sz);
        float f;
        if (is_solid(g, sx, sy, sz)) {
            // half-way bounce-back: the node's own post-collision population
            // along -c arrives back along +c
            float m[10], gg[3];
            load_moments<S>(in, g.N, n, p.inv_scale, m);
#pragma unroll
            for (int a = 0; a < 3; ++a) gg[a] = p.gfield ? p.gfield[a * g.N + n] : p.force[a];
            f = emit_dev<26 - I, ORDER>(node_terms(m, gg), omo_at(p, z));
        } else {
            const long long src = sx + (long long)g.n[0] * (sy + (long long)g.n[1] * sz);
            float m[10], gg[3];
            load_moments<S>(in, g.N, src, p.inv_scale, m);
#pragma unroll
            for (int a = 0; a < 3; ++a) gg[a] = p.gfield ? p.gfield[a * g.N + src] : p.force[a];
            f = emit_dev<I, ORDER>(node_terms(m, gg), omo_at(p, sz));
        }
        acc.template add<I>(f);
    });
    float m[10];
    finalize(acc, m);
    out[n] = S::store(m[0], p.scale[0]);
#pragma unroll
    for (int q = 1; q < 4; ++q) out[q * g.N + n] = S::store(m[q], p.scale[1]);
#pragma unroll
    for (int q = 4; q < 10; ++q) out[q * g.N + n] = S::store(m[q], p.scale[2]);
}

template <class S>
hipError_t launch(const void* in, void* out, const StepParams& p, hipStream_t s) {
    const int block = 256;
    const long long grid = (p.geo.N + block - 1) / block;
    if (p.order == 2)
        hipLaunchKernelGGL((update_direct_kernel<S, 2>), dim3((unsigned)grid), dim3(block), 0, s,
                           (const typename S::T*)in, (typename S::T*)out, p);
    else
        hipLaunchKernelGGL((update_direct_kernel<S, 3>), dim3((unsigned)grid), dim3(block), 0, s,
                           (const typename S::T*)in, (typename S::T*)out, p);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_update_direct(int storage, const void* in, void* out, const StepParams& p, hipStream_t s) {
    switch (storage) {
    case 0: return launch<StoreF32>(in, out, p, s);
    case 1: return launch<StoreF16>(in, out, p, s);
    case 2: return launch<StoreBF16>(in, out, p, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace tslb
