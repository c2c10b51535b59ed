// Device-side building blocks shared by the libnif kernels (gfx950, wave64).
//
//  - pose records and the parameterized deformations D / D^-1 in FP32 (Methodology: rays
//    are traced in deformed space and their samples mapped back to rest space through the
//    inverse deformation);
//  - the FP32 implicit scenes used by rest-space voxelization;
//  - small wave-level helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace nif {

enum { DEF_IDENTITY = 0, DEF_TWIST = 1, DEF_BEND = 2, DEF_TAPER = 3 };

constexpr float kCx = 0.5f, kCy = 0.5f, kCz = 0.5f;   // deformation pivot: cube centre
constexpr float kBinPad = 1e-5f;                      // padding of voxel boxes when binned

// One deformation pose and its deformed-space acceleration grid.
struct PoseDev {
    int32_t kind;
    float s;
    float k0, k1;          // twist: alpha = 0.6 s; bend: kappa = s / 1.5, 1 / kappa; taper: beta = 0.5 s
    float lo[3];           // bin-grid origin (deformed space)
    float bs[3];           // bin size
    float inv_bs[3];
    int32_t nb[3];         // bins per axis
    int32_t empty;         // no occupied voxel
    int32_t pad;
    int64_t vert_off;      // into the vertex array, (N+1)^3 float4 per pose
    int64_t bin_off;       // into bin_start, nbins + 1 per pose
    int64_t ref_off;       // into bin_cells
};

// The deformation and its inverse are evaluated with FP contraction off: every kernel that
// places lattice vertices or maps points must round identically, whatever the surrounding code.
#pragma clang fp contract(off)
__host__ __device__ inline void pose_constants(int kind, float s, float* k0, float* k1) {
    *k0 = 0.f; *k1 = 0.f;
    if (kind == DEF_TWIST) *k0 = 0.6f * s;
    if (kind == DEF_BEND) { *k0 = s / 1.5f; *k1 = s > 0.f ? 1.5f / s : 0.f; }
    if (kind == DEF_TAPER) *k0 = 0.5f * s;
}

// Rest -> deformed.  Used to build the deformed lattice vertices.
__device__ inline float3 deform(const PoseDev& P, float3 p) {
    float3 q = p;
    if (P.kind == DEF_TWIST) {
        float sn, cs;
        sincosf(P.k0 * p.z, &sn, &cs);
        float x = p.x - kCx, y = p.y - kCy;
        q.x = kCx + (cs * x - sn * y);
        q.y = kCy + (sn * x + cs * y);
    } else if (P.kind == DEF_BEND && P.k0 > 0.f) {
        float u = p.x - kCx;
        float ph = P.k0 * (p.z - kCz);
        float sn, cs;
        sincosf(ph, &sn, &cs);
        // x' = cx + u cos(ph) + (1 - cos ph) / kappa, with 1 - cos = 2 sin^2(ph/2) to avoid
        // cancellation for small angles; z' = cz + (1/kappa - u) sin(ph)
        float sh = sinf(0.5f * ph);
        q.x = kCx + u * cs + 2.f * sh * sh * P.k1;
        q.z = kCz + (P.k1 - u) * sn;
    } else if (P.kind == DEF_TAPER) {
        float sg = 1.f - P.k0 * p.z;
        q.x = kCx + sg * (p.x - kCx);
        q.y = kCy + sg * (p.y - kCy);
    }
    return q;
}

// Deformed -> rest (the analytic inverse).
__device__ inline float3 deform_inv(const PoseDev& P, float3 q) {
    float3 p = q;
    if (P.kind == DEF_TWIST) {
        float sn, cs;
        sincosf(P.k0 * q.z, &sn, &cs);
        float x = q.x - kCx, y = q.y - kCy;
        p.x = kCx + (cs * x + sn * y);
        p.y = kCy + (-sn * x + cs * y);
    } else if (P.kind == DEF_BEND && P.k0 > 0.f) {
        // With X = x' - cx, Z = z' - cz and kappa = k: the rest offset u = 1/k - rho where
        // rho = |(1/k - X, Z)|.  Written without the cancellation of 1/k - rho:
        //   u = (2X - k (X^2 + Z^2)) / (1 + k rho),  k rho = |(1 - k X, k Z)|,
        //   z = cz + atan2(k Z, 1 - k X) / k.
        float X = q.x - kCx, Z = q.z - kCz, k = P.k0;
        float a = 1.f - k * X, b = k * Z;
        float krho = sqrtf(a * a + b * b);
        p.x = kCx + (2.f * X - k * (X * X + Z * Z)) / (1.f + krho);
        p.z = kCz + atan2f(b, a) * P.k1;
    } else if (P.kind == DEF_TAPER) {
        float sg = 1.f - P.k0 * q.z;
        p.x = kCx + (q.x - kCx) / sg;
        p.y = kCy + (q.y - kCy) / sg;
    }
    return p;
}

// Normal of the deformed surface at D(p) from the rest-space normal n at p: (dD/dp)^-T n,
// normalized.  With the Jacobian's columns a, b, c, J^-T n is proportional to
// n.x (b x c) + n.y (c x a) + n.z (a x b) (the cofactor rows; det J > 0 for every pose).
__device__ inline float3 deform_normal(const PoseDev& P, float3 p, float3 n) {
    float3 a = make_float3(1.f, 0.f, 0.f), b = make_float3(0.f, 1.f, 0.f), c = make_float3(0.f, 0.f, 1.f);
    if (P.kind == DEF_TWIST) {
        float sn, cs;
        sincosf(P.k0 * p.z, &sn, &cs);
        const float u = p.x - kCx, v = p.y - kCy;
        a = make_float3(cs, sn, 0.f);
        b = make_float3(-sn, cs, 0.f);
        c = make_float3(P.k0 * (-sn * u - cs * v), P.k0 * (cs * u - sn * v), 1.f);
    } else if (P.kind == DEF_BEND && P.k0 > 0.f) {
        float sn, cs;
        sincosf(P.k0 * (p.z - kCz), &sn, &cs);
        const float w = 1.f - P.k0 * (p.x - kCx);
        a = make_float3(cs, 0.f, -sn);
        c = make_float3(sn * w, 0.f, cs * w);
    } else if (P.kind == DEF_TAPER) {
        const float sg = 1.f - P.k0 * p.z;
        a = make_float3(sg, 0.f, 0.f);
        b = make_float3(0.f, sg, 0.f);
        c = make_float3(-P.k0 * (p.x - kCx), -P.k0 * (p.y - kCy), 1.f);
    }
    const float3 bc = make_float3(b.y * c.z - b.z * c.y, b.z * c.x - b.x * c.z, b.x * c.y - b.y * c.x);
    const float3 ca = make_float3(c.y * a.z - c.z * a.y, c.z * a.x - c.x * a.z, c.x * a.y - c.y * a.x);
    const float3 ab = make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
    float3 m = make_float3(n.x * bc.x + n.y * ca.x + n.z * ab.x, n.x * bc.y + n.y * ca.y + n.z * ab.y,
                           n.x * bc.z + n.y * ca.z + n.z * ab.z);
    const float l = sqrtf(m.x * m.x + m.y * m.y + m.z * m.z);
    const float il = l > 0.f ? 1.f / l : 0.f;
    return make_float3(m.x * il, m.y * il, m.z * il);
}

// ------------------------------------------------------------------ implicit scenes (FP32)
enum { SCENE_TORUS = 0, SCENE_SPHERES = 1, SCENE_BLOBS = 2 };
constexpr int kSceneStride = 8;

#pragma clang fp contract(fast)

__device__ inline float scene_f(int kind, const float* sp, float3 p) {
    if (kind == SCENE_TORUS) {
        float dx = p.x - sp[0], dy = p.y - sp[1], dz = p.z - sp[2];
        float q = sqrtf(dx * dx + dy * dy) - sp[3];
        return q * q + dz * dz - sp[4] * sp[4];
    }
    int n = (int)sp[0];
    if (kind == SCENE_SPHERES) {
        float best = INFINITY;
        for (int i = 0; i < n; ++i) {
            const float* c = sp + 1 + kSceneStride * i;
            float dx = p.x - c[0], dy = p.y - c[1], dz = p.z - c[2];
            best = fminf(best, sqrtf(dx * dx + dy * dy + dz * dz) - c[3]);
        }
        return best;
    }
    float g = 0.f;
    for (int i = 0; i < n; ++i) {
        const float* b = sp + 1 + kSceneStride * i;
        float dx = p.x - b[0], dy = p.y - b[1], dz = p.z - b[2];
        g += expf(-(dx * dx + dy * dy + dz * dz) / (2.f * b[3] * b[3]));
    }
    return 0.5f - g;
}

// ------------------------------------------------------------------ wave helpers
__device__ inline int lane_id() { return __lane_id(); }

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

__device__ inline int popc64(uint64_t m) { return __popcll(m); }

// Number of set bits of m below this lane.
__device__ inline int rank_below(uint64_t m) {
    return __popcll(m & ((1ull << lane_id()) - 1ull));
}

}  // namespace nif
