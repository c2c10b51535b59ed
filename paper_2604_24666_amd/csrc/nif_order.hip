// Spatial ordering of a training batch.  The batch's samples are stably sorted by the Morton
// code of their rest-space entry point (10 bits per axis) before the step, so that the waves
// of the forward touch neighbouring table lines and the fill writes runs of additions to the
// same buckets.  The step's results are sums over the samples, so the order changes only
// their rounding (the table gradient, summed in fixed point, not at all); the radix sort is
// stable, so the step stays deterministic.
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "nif_internal.hpp"

namespace nif {

__device__ __forceinline__ uint32_t spread3(uint32_t v) {     // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_morton_keys(const float* __restrict__ x0, int64_t B, uint32_t* __restrict__ key,
                              uint32_t* __restrict__ idx) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < B; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c = 0;
        for (int a = 0; a < 3; ++a) {
            const float v = fminf(fmaxf(x0[a * B + i], 0.f), 1.f);
            c |= spread3((uint32_t)(v * 1023.f)) << a;
        }
        key[i] = c;
        idx[i] = (uint32_t)i;
    }
}

// out[k] = in[order[k]] for every array of the batch (SoA [3][B] for points, normals, albedo).
__global__ void k_permute_batch(nif_batch in, nif_batch out, const uint32_t* __restrict__ order, int64_t B) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < B; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = order[k];
        for (int a = 0; a < 3; ++a) {
            const_cast<float*>(out.x0)[a * B + k] = in.x0[a * B + i];
            const_cast<float*>(out.x1)[a * B + k] = in.x1[a * B + i];
            const_cast<float*>(out.n)[a * B + k] = in.n[a * B + i];
            const_cast<float*>(out.a)[a * B + k] = in.a[a * B + i];
        }
        const_cast<uint8_t*>(out.hit)[k] = in.hit[i];
        const_cast<float*>(out.t)[k] = in.t[i];
        const_cast<int32_t*>(out.m)[k] = in.m[i];
    }
}

size_t order_temp_bytes(int64_t B) {
    size_t bytes = 0;
    if (rocprim::radix_sort_pairs(nullptr, bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                  (uint32_t*)nullptr, (size_t)B, 0u, 30u) != hipSuccess)
        return 0;
    return bytes;
}

int order_batch(nif_model* m, const nif_batch* b, int64_t B, nif_batch* sorted, hipStream_t st) {
    uint32_t* key = m->ord_u32;
    uint32_t* key2 = key + m->max_batch;
    uint32_t* idx = key2 + m->max_batch;
    uint32_t* idx2 = idx + m->max_batch;
    const int64_t grid = std::min<int64_t>((B + 255) / 256, 4096);
    hipLaunchKernelGGL(k_morton_keys, dim3((unsigned)grid), dim3(256), 0, st, b->x0, B, key, idx);
    size_t bytes = m->ord_temp_bytes;
    int rc = check_hip(rocprim::radix_sort_pairs(m->ord_temp, bytes, key, key2, idx, idx2, (size_t)B, 0u, 30u, st),
                       "batch ordering sort");
    if (rc) return rc;
    nif_batch s;
    s.x0 = m->ord_f32;
    s.x1 = m->ord_f32 + 3 * B;
    s.n = m->ord_f32 + 6 * B;
    s.a = m->ord_f32 + 9 * B;
    s.t = m->ord_f32 + 12 * B;
    s.m = reinterpret_cast<const int32_t*>(m->ord_f32 + 13 * B);
    s.hit = reinterpret_cast<const uint8_t*>(m->ord_f32 + 14 * B);
    hipLaunchKernelGGL(k_permute_batch, dim3((unsigned)grid), dim3(256), 0, st, *b, s, idx2, B);
    *sorted = s;
    return check_hip(hipGetLastError(), "batch ordering");
}

}  // namespace nif
