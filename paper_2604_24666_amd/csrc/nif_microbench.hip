// Device ceilings for the rooflines the measurements are reported against (not part of the
// method): streaming HBM reads, random gathers of table-sized entries from a table of a given
// size (the access pattern of the hash-grid lookups: a 32 MiB FP16 table fits the Infinity
// Cache but not an XCD's L2), and the MFMA rates of the instruction forms the kernels use.
#include "nif_internal.hpp"
#include "nif_net.hpp"

namespace nif {

namespace {

// Streaming read of n float4 (grid-stride), reduced to one value per thread so the loads stay.
__global__ void __launch_bounds__(256) k_mb_stream(const float4* __restrict__ a, int64_t n, float* __restrict__ sink) {
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float4 v = a[i];
        s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
    }
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s.x + s.y + s.z + s.w;
}

__device__ __forceinline__ uint32_t mb_hash(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

// Random gathers: every thread issues `per_thread` loads of E-byte entries (E = 4: one half2
// table entry; 8: an aligned pair of them) at hashed indices into a table of n_entries, eight at
// a time so that eight are in flight per lane (as a lookup batch keeps its corners in flight).
template <typename E>
__global__ void __launch_bounds__(256) k_mb_gather(const E* __restrict__ tab, uint32_t n_entries, int32_t per_thread,
                                                   uint32_t salt, float* __restrict__ sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (int32_t i = 0; i < per_thread; i += 8) {
        E v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = tab[mb_hash(tid * 0x9e3779b9u + (uint32_t)(i + k) * 0x85ebca6bu + salt) % n_entries];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if constexpr (sizeof(E) == 4) acc += v[k];
            else acc += v[k].x ^ v[k].y;
        }
    }
    sink[tid] = (float)acc;
}

// MFMA rate: four independent accumulator chains per wave, `iters` rounds of each chain.
template <int FORM>
__global__ void __launch_bounds__(256) k_mb_mfma(int32_t iters, float seed, float* __restrict__ sink) {
    floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0, c2 = c0, c3 = c0;
    const float a = seed * (float)(threadIdx.x & 7), b = seed * (float)(threadIdx.x >> 3);
    if constexpr (FORM == 0) {                      // v_mfma_f32_16x16x4_f32
        for (int32_t i = 0; i < iters; ++i) {
            c0 = mfma32(a, b, c0); c1 = mfma32(b, a, c1); c2 = mfma32(a, a, c2); c3 = mfma32(b, b, c3);
        }
    } else {                                        // v_mfma_f32_16x16x16_bf16
        const shortx4 pa = pack4<P_BF16>(a, b, a, b), pb = pack4<P_BF16>(b, a, b, a);
        for (int32_t i = 0; i < iters; ++i) {
            c0 = mfma16<P_BF16>(pa, pb, c0); c1 = mfma16<P_BF16>(pb, pa, c1);
            c2 = mfma16<P_BF16>(pa, pa, c2); c3 = mfma16<P_BF16>(pb, pb, c3);
        }
    }
    const floatx4 s = c0 + c1 + c2 + c3;
    sink[blockIdx.x * blockDim.x + threadIdx.x] = s[0] + s[1] + s[2] + s[3];
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

int microbench(int32_t kind, int64_t n_bytes, int64_t n_ops, int32_t reps, double* result, hipStream_t st) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const unsigned blocks = (unsigned)cus * 16, threads = 256;
    DevBuf buf, sink;
    if (kind <= 2 && hipMalloc(&buf.p, (size_t)n_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(NIF_E_OOM, "microbenchmark buffer allocation failed");
    }
    if (hipMalloc(&sink.p, sizeof(float) * (size_t)blocks * threads) != hipSuccess) {
        (void)hipGetLastError();
        return fail(NIF_E_OOM, "microbenchmark buffer allocation failed");
    }
    if (kind <= 2) {
        int rc = check_hip(hipMemsetAsync(buf.p, 0, (size_t)n_bytes, st), "microbenchmark fill");
        if (rc) return rc;
    }
    float* snk = static_cast<float*>(sink.p);
    const int64_t total_threads = (int64_t)blocks * threads;
    // per-thread work of the gathers and the MFMA loop, rounded so the totals are exact
    const int32_t per_thread = (int32_t)std::max<int64_t>(8, (n_ops / total_threads + 7) / 8 * 8);
    const int32_t iters = (int32_t)std::max<int64_t>(1, n_ops / (total_threads / 64) / 4);
    auto launch = [&](uint32_t salt) {
        switch (kind) {
            case 0: hipLaunchKernelGGL(k_mb_stream, dim3(blocks), dim3(threads), 0, st,
                                       static_cast<const float4*>(buf.p), n_bytes / 16, snk); break;
            case 1: hipLaunchKernelGGL(k_mb_gather<uint32_t>, dim3(blocks), dim3(threads), 0, st,
                                       static_cast<const uint32_t*>(buf.p), (uint32_t)(n_bytes / 4), per_thread, salt, snk); break;
            case 2: hipLaunchKernelGGL(k_mb_gather<uint2>, dim3(blocks), dim3(threads), 0, st,
                                       static_cast<const uint2*>(buf.p), (uint32_t)(n_bytes / 8), per_thread, salt, snk); break;
            case 3: hipLaunchKernelGGL(k_mb_mfma<0>, dim3(blocks), dim3(threads), 0, st, iters, 1e-3f * (float)(salt + 1), snk); break;
            default: hipLaunchKernelGGL(k_mb_mfma<1>, dim3(blocks), dim3(threads), 0, st, iters, 1e-3f * (float)(salt + 1), snk); break;
        }
    };
    hipEvent_t e0, e1;
    int rc = check_hip(hipEventCreate(&e0), "event");
    if (rc) return rc;
    if ((rc = check_hip(hipEventCreate(&e1), "event"))) { (void)hipEventDestroy(e0); return rc; }
    launch(0);                                                  // warm-up
    (void)hipEventRecord(e0, st);
    for (int32_t r = 0; r < reps; ++r) launch((uint32_t)r + 1);
    (void)hipEventRecord(e1, st);
    rc = check_hip(hipEventSynchronize(e1), "microbenchmark");
    float ms = 0.f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) rc = check_hip(hipGetLastError(), "microbenchmark launch");
    if (rc) return rc;
    const double sec = (double)ms * 1e-3 / reps;
    double work;
    switch (kind) {
        case 0: work = (double)(n_bytes / 16 * 16); break;                               // bytes read
        case 1: work = (double)total_threads * per_thread * 4.0; break;                 // bytes gathered
        case 2: work = (double)total_threads * per_thread * 8.0; break;
        case 3: work = (double)(total_threads / 64) * iters * 4.0 * 2048.0; break;      // FLOP
        default: work = (double)(total_threads / 64) * iters * 4.0 * 8192.0; break;
    }
    result[0] = work / sec;
    result[1] = sec * 1e3;
    return NIF_OK;
}

}  // namespace nif
