// Ground-truth labels of rest-space segments on the GPU (training-data generation).
//
// Methodology, the local linear approximation: every deformed ray segment is represented by
// its rest-space chord [x0, x1], and the network is supervised with the rest geometry met
// along that chord: occlusion, distance from x0 to the first surface point, the surface
// normal there, albedo and material.  The rest geometry here is an implicit scene f (f < 0
// inside; torus, union of spheres, Gaussian blobs, parameters as for nif_voxelize).
//
// The first point of the chord with f <= 0: t = 0 if f(x0) <= 0; for spheres the entering
// root of each sphere's quadratic (the smallest in [0, len]); otherwise 256 uniform sign steps
// over [0, len] and bisection of the first bracket down to 1e-13.  Normal = grad f / |grad f|
// at that point.  Everything in FP64, so the sign decisions are taken in the same precision as
// the reference implementation.
#include <cmath>
#include <mutex>
#include <vector>

#include "nif_internal.hpp"

namespace nif {

// FP64 without contraction into FMA, so that the sign decisions round like plain IEEE code.
#pragma clang fp contract(off)

__device__ double scene_value(int kind, const double* __restrict__ sp, const double p[3]) {
    if (kind == 0) {
        const double dx = p[0] - sp[0], dy = p[1] - sp[1], dz = p[2] - sp[2];
        const double q = sqrt(dx * dx + dy * dy) - sp[3];
        return q * q + dz * dz - sp[4] * sp[4];
    }
    const int n = (int)sp[0];
    if (kind == 1) {
        double best = INFINITY;
        for (int i = 0; i < n; ++i) {
            const double* c = sp + 1 + kSceneStride * i;
            const double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
            best = fmin(best, sqrt(dx * dx + dy * dy + dz * dz) - c[3]);
        }
        return best;
    }
    double g = 0.0;
    for (int i = 0; i < n; ++i) {
        const double* b = sp + 1 + kSceneStride * i;
        const double dx = p[0] - b[0], dy = p[1] - b[1], dz = p[2] - b[2];
        g += exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * b[3] * b[3]));
    }
    return 0.5 - g;
}

// Index of the sphere with the smallest signed distance at p.
__device__ int nearest_sphere(const double* __restrict__ sp, const double p[3]) {
    const int n = (int)sp[0];
    double best = INFINITY;
    int arg = 0;
    for (int i = 0; i < n; ++i) {
        const double* c = sp + 1 + kSceneStride * i;
        const double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
        const double v = sqrt(dx * dx + dy * dy + dz * dz) - c[3];
        if (v < best) { best = v; arg = i; }
    }
    return arg;
}

__device__ void scene_gradient(int kind, const double* __restrict__ sp, const double p[3], double g[3]) {
    if (kind == 0) {
        const double dx = p[0] - sp[0], dy = p[1] - sp[1], dz = p[2] - sp[2];
        const double rho = sqrt(dx * dx + dy * dy);
        const double k = rho > 0.0 ? 2.0 * (rho - sp[3]) / rho : 0.0;
        g[0] = k * dx; g[1] = k * dy; g[2] = 2.0 * dz;
        return;
    }
    if (kind == 1) {
        const double* c = sp + 1 + kSceneStride * nearest_sphere(sp, p);
        const double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r == 0.0) { g[0] = 0.0; g[1] = 0.0; g[2] = 1.0; return; }
        g[0] = dx / r; g[1] = dy / r; g[2] = dz / r;
        return;
    }
    const int n = (int)sp[0];
    g[0] = g[1] = g[2] = 0.0;
    for (int i = 0; i < n; ++i) {
        const double* b = sp + 1 + kSceneStride * i;
        const double dx = p[0] - b[0], dy = p[1] - b[1], dz = p[2] - b[2];
        const double s2 = b[3] * b[3];
        const double e = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s2));
        g[0] += e * dx / s2; g[1] += e * dy / s2; g[2] += e * dz / s2;
    }
}

__device__ void scene_attributes(int kind, const double* __restrict__ sp, const double p[3], double a[3], int* mat) {
    if (kind == 0) {
        for (int c = 0; c < 3; ++c) a[c] = 0.5 + 0.4 * sin(2.0 * M_PI * (2.0 * p[c] + c / 3.0));
        *mat = p[0] >= 0.5 ? 1 : 0;
        return;
    }
    if (kind == 1) {
        const double* c = sp + 1 + kSceneStride * nearest_sphere(sp, p);
        a[0] = c[4]; a[1] = c[5]; a[2] = c[6];
        *mat = (int)c[7];
        return;
    }
    const int n = (int)sp[0];
    double wsum = 0.0, wbest = -1.0;
    int arg = 0;
    a[0] = a[1] = a[2] = 0.0;
    for (int i = 0; i < n; ++i) {
        const double* b = sp + 1 + kSceneStride * i;
        const double dx = p[0] - b[0], dy = p[1] - b[1], dz = p[2] - b[2];
        const double e = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * b[3] * b[3]));
        wsum += e;
        a[0] += e * b[4]; a[1] += e * b[5]; a[2] += e * b[6];
        if (e > wbest) { wbest = e; arg = i; }
    }
    if (wsum > 0.0) { a[0] /= wsum; a[1] /= wsum; a[2] /= wsum; }
    *mat = (int)sp[1 + kSceneStride * arg + 7];
}

// First parameter tau in [0, len] of x0 + tau u with f <= 0.
__device__ bool chord_first_inside(int kind, const double* __restrict__ sp, int force_march, const double x0[3],
                                   const double u[3], double len, double* tau) {
    if (scene_value(kind, sp, x0) <= 0.0) { *tau = 0.0; return true; }
    if (len <= 0.0) return false;
    if (kind == 1 && !force_march) {
        const int n = (int)sp[0];
        double best = INFINITY;
        for (int i = 0; i < n; ++i) {
            const double* c = sp + 1 + kSceneStride * i;
            const double w[3] = {x0[0] - c[0], x0[1] - c[1], x0[2] - c[2]};
            const double b = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
            const double disc = b * b - (w[0] * w[0] + w[1] * w[1] + w[2] * w[2] - c[3] * c[3]);
            if (disc < 0.0) continue;
            const double r = -b - sqrt(disc);          // entering root (x0 is outside every sphere)
            if (r >= 0.0 && r <= len && r < best) best = r;
        }
        if (best < INFINITY) { *tau = best; return true; }
        return false;
    }
    constexpr int kSteps = 256;
    double prev = 0.0;
    for (int s = 1; s <= kSteps; ++s) {
        const double t = len * s / kSteps;
        const double p[3] = {x0[0] + t * u[0], x0[1] + t * u[1], x0[2] + t * u[2]};
        if (scene_value(kind, sp, p) <= 0.0) {
            double a = prev, b = t;                     // f(a) > 0 >= f(b)
            while (b - a > 1e-13) {
                const double m = 0.5 * (a + b);
                const double q[3] = {x0[0] + m * u[0], x0[1] + m * u[1], x0[2] + m * u[2]};
                if (scene_value(kind, sp, q) <= 0.0) b = m; else a = m;
            }
            *tau = b;
            return true;
        }
        prev = t;
    }
    return false;
}

__global__ void __launch_bounds__(256) k_label(int kind, const double* __restrict__ sp, int force_march,
                                               const float* __restrict__ x0, const float* __restrict__ x1, int64_t n,
                                               uint8_t* __restrict__ hit, float* __restrict__ t, float* __restrict__ nrm,
                                               float* __restrict__ alb, int32_t* __restrict__ mat) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double p0[3] = {x0[i], x0[n + i], x0[2 * n + i]};
        const double e[3] = {(double)x1[i] - p0[0], (double)x1[n + i] - p0[1], (double)x1[2 * n + i] - p0[2]};
        const double len = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        double u[3] = {0.0, 0.0, 0.0};
        if (len > 0.0) { u[0] = e[0] / len; u[1] = e[1] / len; u[2] = e[2] / len; }
        double tau = 0.0;
        const bool h = chord_first_inside(kind, sp, force_march, p0, u, len, &tau);
        double g[3] = {0.0, 0.0, 0.0}, a[3] = {0.0, 0.0, 0.0};
        int m = 0;
        if (h) {
            const double p[3] = {p0[0] + tau * u[0], p0[1] + tau * u[1], p0[2] + tau * u[2]};
            scene_gradient(kind, sp, p, g);
            const double gl = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            if (gl > 0.0) { g[0] /= gl; g[1] /= gl; g[2] /= gl; }
            else { g[0] = g[1] = g[2] = 0.0; }
            scene_attributes(kind, sp, p, a, &m);
        } else {
            tau = 0.0;
        }
        if (hit) hit[i] = h ? 1 : 0;
        if (t) t[i] = (float)tau;
        if (nrm) { nrm[i] = (float)g[0]; nrm[n + i] = (float)g[1]; nrm[2 * n + i] = (float)g[2]; }
        if (alb) { alb[i] = (float)a[0]; alb[n + i] = (float)a[1]; alb[2 * n + i] = (float)a[2]; }
        if (mat) mat[i] = m;
    }
}

static void launch_label(int kind, const double* sp_dev, int force_march, const float* x0, const float* x1, int64_t n,
                         uint8_t* hit, float* t, float* nrm, float* alb, int32_t* mat, hipStream_t st) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)cus * 16);
    hipLaunchKernelGGL(k_label, dim3((unsigned)blocks), dim3(256), 0, st, kind, sp_dev, force_march, x0, x1, n, hit, t,
                       nrm, alb, mat);
}

int label_launch(int kind, const double* params_host, int32_t n_params, int force_march, const float* x0,
                 const float* x1, int64_t n, uint8_t* hit, float* t, float* nrm, float* alb, int32_t* mat,
                 hipStream_t st) {
    if (n == 0) return NIF_OK;
    double* dp = nullptr;
    int rc = check_hip(hipMalloc(&dp, sizeof(double) * n_params), "hipMalloc scene");
    if (rc) return rc;
    rc = check_hip(hipMemcpyAsync(dp, params_host, sizeof(double) * n_params, hipMemcpyHostToDevice, st), "copy scene");
    if (!rc) {
        launch_label(kind, dp, force_march, x0, x1, n, hit, t, nrm, alb, mat, st);
        rc = check_hip(hipGetLastError(), "k_label launch");
    }
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "label sync");
    (void)hipFree(dp);
    return rc;
}

// Allocation-free labelling: the scene parameters are staged in a per-device array of the
// code object instead of a buffer allocated per call.  The array's host-side name is not a
// device address; its address on each device comes from hipGetSymbolAddress, once per device,
// with that device current, and only that address is handed to copies and kernels.  Every
// call on a device shares its array: calls that overlap on one device (other streams, other
// threads) race on it.
static __device__ __align__(256) double scratch[kLabelScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

static int label_scratch(double** out) {
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return fail(NIF_E_DEVICE, "device index beyond the library's table of 64");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if ((rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))) return rc;
        if (!p) return fail(NIF_E_DEVICE, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return NIF_OK;
}

int label_launch_noalloc(int kind, const double* params_host, int32_t n_params, int force_march, const float* x0,
                         const float* x1, int64_t n, uint8_t* hit, float* t, float* nrm, float* alb, int32_t* mat,
                         hipStream_t st) {
    if (n_params > kLabelScratchDoubles)
        return fail(NIF_E_INVALID_ARG, "n_params exceeds the allocation-free label scratch (4104 values)");
    if (n == 0) return NIF_OK;
    double* sp = nullptr;
    int rc = label_scratch(&sp);
    if (rc) return rc;
    rc = check_hip(hipMemcpyAsync(sp, params_host, sizeof(double) * n_params, hipMemcpyHostToDevice, st),
                   "stage scene parameters");
    if (rc) return rc;
    launch_label(kind, sp, force_march, x0, x1, n, hit, t, nrm, alb, mat, st);
    return check_hip(hipGetLastError(), "k_label launch");
}

#pragma clang fp contract(fast)

}  // namespace nif
