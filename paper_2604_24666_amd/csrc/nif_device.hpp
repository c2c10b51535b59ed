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

enum { DEF_IDENTITY = 0, DEF_TWIST = 1, DEF_BEND = 2, DEF_TAPER = 3, DEF_TWIST_BEND = 4 };

constexpr float kCx = 0.5f, kCy = 0.5f, kCz = 0.5f;   // deformation pivot: cube centre
constexpr float kBinPad = 1e-5f;                      // padding of voxel boxes when binned

// One deformation pose and its deformed-space acceleration grid.
struct PoseDev {
    int32_t kind;
    float s;
    float k0, k1;          // twist: alpha = 0.6 s; bend: kappa = s / 1.5, 1 / kappa; taper: beta = 0.5 s;
                           // twist-bend: alpha, kappa (and k2 = 1 / kappa)
    float lo[3];           // bin-grid origin (deformed space)
    float bs[3];           // bin size
    float inv_bs[3];
    int32_t nb[3];         // bins per axis
    int32_t empty;         // no occupied voxel
    float k2;
    int64_t vert_off;      // into the vertex array, (N+1)^3 float4 per pose
    int64_t bin_off;       // into bin_start, nbins + 1 per pose
    int64_t ref_off;       // into bin_cells
};

// The deformation and its inverse are evaluated with FP contraction off: every kernel that
// places lattice vertices or maps points must round identically, whatever the surrounding code.
#pragma clang fp contract(off)
__host__ __device__ inline void pose_constants(int kind, float s, float* k0, float* k1, float* k2) {
    *k0 = 0.f; *k1 = 0.f; *k2 = 0.f;
    if (kind == DEF_TWIST) *k0 = 0.6f * s;
    if (kind == DEF_BEND) { *k0 = s / 1.5f; *k1 = s > 0.f ? 1.5f / s : 0.f; }
    if (kind == DEF_TAPER) *k0 = 0.5f * s;
    if (kind == DEF_TWIST_BEND) { *k0 = 0.6f * s; *k1 = s / 1.5f; *k2 = s > 0.f ? 1.5f / s : 0.f; }
}

// The elementary deformations (alpha, kappa, 1/kappa, beta as in pose_constants).
__device__ inline float3 twist_fwd(float al, float3 p) {
    float sn, cs;
    sincosf(al * p.z, &sn, &cs);
    const float x = p.x - kCx, y = p.y - kCy;
    return make_float3(kCx + (cs * x - sn * y), kCy + (sn * x + cs * y), p.z);
}
__device__ inline float3 twist_inv(float al, float3 q) {
    float sn, cs;
    sincosf(al * q.z, &sn, &cs);
    const float x = q.x - kCx, y = q.y - kCy;
    return make_float3(kCx + (cs * x + sn * y), kCy + (-sn * x + cs * y), q.z);
}
__device__ inline float3 bend_fwd(float k, float ik, float3 p) {
    if (!(k > 0.f)) return p;
    const float u = p.x - kCx;
    const float ph = k * (p.z - kCz);
    float sn, cs;
    sincosf(ph, &sn, &cs);
    // x' = cx + u cos(ph) + (1 - cos ph) / kappa, with 1 - cos = 2 sin^2(ph/2) to avoid
    // cancellation for small angles; z' = cz + (1/kappa - u) sin(ph)
    const float sh = sinf(0.5f * ph);
    return make_float3(kCx + u * cs + 2.f * sh * sh * ik, p.y, kCz + (ik - u) * sn);
}
__device__ inline float3 bend_inv(float k, float ik, float3 q) {
    if (!(k > 0.f)) return q;
    // With X = x' - cx, Z = z' - cz: the rest offset u = 1/k - rho where rho = |(1/k - X, Z)|.
    // Written without the cancellation of 1/k - rho:
    //   u = (2X - k (X^2 + Z^2)) / (1 + k rho),  k rho = |(1 - k X, k Z)|,
    //   z = cz + atan2(k Z, 1 - k X) / k.
    const float X = q.x - kCx, Z = q.z - kCz;
    const float a = 1.f - k * X, b = k * Z;
    const float krho = sqrtf(a * a + b * b);
    return make_float3(kCx + (2.f * X - k * (X * X + Z * Z)) / (1.f + krho), q.y, kCz + atan2f(b, a) * ik);
}
__device__ inline float3 taper_fwd(float be, float3 p) {
    const float sg = 1.f - be * p.z;
    return make_float3(kCx + sg * (p.x - kCx), kCy + sg * (p.y - kCy), p.z);
}
__device__ inline float3 taper_inv(float be, float3 q) {
    const float sg = 1.f - be * q.z;
    return make_float3(kCx + (q.x - kCx) / sg, kCy + (q.y - kCy) / sg, q.z);
}

// Rest -> deformed.  Used to build the deformed lattice vertices.
__device__ inline float3 deform(const PoseDev& P, float3 p) {
    if (P.kind == DEF_TWIST) return twist_fwd(P.k0, p);
    if (P.kind == DEF_BEND) return bend_fwd(P.k0, P.k1, p);
    if (P.kind == DEF_TAPER) return taper_fwd(P.k0, p);
    if (P.kind == DEF_TWIST_BEND) return bend_fwd(P.k1, P.k2, twist_fwd(P.k0, p));
    return p;
}

// Deformed -> rest (the analytic inverse).
__device__ inline float3 deform_inv(const PoseDev& P, float3 q) {
    if (P.kind == DEF_TWIST) return twist_inv(P.k0, q);
    if (P.kind == DEF_BEND) return bend_inv(P.k0, P.k1, q);
    if (P.kind == DEF_TAPER) return taper_inv(P.k0, q);
    if (P.kind == DEF_TWIST_BEND) return twist_inv(P.k0, bend_inv(P.k1, P.k2, q));
    return q;
}

// (dD/dp)^-T n up to a positive factor for one elementary deformation at p.  With the
// Jacobian's columns a, b, c it is n.x (b x c) + n.y (c x a) + n.z (a x b) (the cofactor
// rows; det J > 0 for every pose).
__device__ inline float3 cofactor_apply(float3 a, float3 b, float3 c, float3 n) {
    const float3 bc = make_float3(b.y * c.z - b.z * c.y, b.z * c.x - b.x * c.z, b.x * c.y - b.y * c.x);
    const float3 ca = make_float3(c.y * a.z - c.z * a.y, c.z * a.x - c.x * a.z, c.x * a.y - c.y * a.x);
    const float3 ab = make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
    return make_float3(n.x * bc.x + n.y * ca.x + n.z * ab.x, n.x * bc.y + n.y * ca.y + n.z * ab.y,
                       n.x * bc.z + n.y * ca.z + n.z * ab.z);
}
__device__ inline float3 twist_normal(float al, float3 p, float3 n) {
    float sn, cs;
    sincosf(al * p.z, &sn, &cs);
    const float u = p.x - kCx, v = p.y - kCy;
    return cofactor_apply(make_float3(cs, sn, 0.f), make_float3(-sn, cs, 0.f),
                          make_float3(al * (-sn * u - cs * v), al * (cs * u - sn * v), 1.f), n);
}
__device__ inline float3 bend_normal(float k, float3 p, float3 n) {
    if (!(k > 0.f)) return n;
    float sn, cs;
    sincosf(k * (p.z - kCz), &sn, &cs);
    const float w = 1.f - k * (p.x - kCx);
    return cofactor_apply(make_float3(cs, 0.f, -sn), make_float3(0.f, 1.f, 0.f), make_float3(sn * w, 0.f, cs * w), n);
}
__device__ inline float3 taper_normal(float be, float3 p, float3 n) {
    const float sg = 1.f - be * p.z;
    return cofactor_apply(make_float3(sg, 0.f, 0.f), make_float3(0.f, sg, 0.f),
                          make_float3(-be * (p.x - kCx), -be * (p.y - kCy), 1.f), n);
}

// Normal of the deformed surface at D(p) from the rest-space normal n at p: (dD/dp)^-T n,
// normalized (a composed pose applies the factors' transforms in turn, each at its own point).
__device__ inline float3 deform_normal(const PoseDev& P, float3 p, float3 n) {
    float3 m = n;
    if (P.kind == DEF_TWIST) m = twist_normal(P.k0, p, n);
    else if (P.kind == DEF_BEND) m = bend_normal(P.k0, p, n);
    else if (P.kind == DEF_TAPER) m = taper_normal(P.k0, p, n);
    else if (P.kind == DEF_TWIST_BEND) m = bend_normal(P.k1, twist_fwd(P.k0, p), twist_normal(P.k0, p, n));
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
