// Ray traversal through the occupied deformed voxels of one pose (FP32).
//
// Methodology, "Voxel Traversal under Deformation" and "Segmented Ray Distance
// Accumulation": a straight deformed-space ray crosses a sequence of deformed voxels; every
// occupied one contributes an entry/exit pair.  A deformed voxel is the hexahedron of its 8
// deformed lattice vertices with each face split along its main diagonal (the same two
// triangles for both voxels sharing the face), so the lattice is watertight.
//
// Exact voxel test.  The line o + t d crosses triangle (A, B, C) iff the three signed
// volumes d . ((P - o) x (Q - o)) of its edges have one sign.  Each of the 18 edges of a
// voxel (12 outer, 6 face diagonals) gets one sign computed for its canonical orientation
// (lower vertex first; an exact zero counts as positive) and negated for the other
// orientation, so every crossing decision is consistent between the two triangles of a
// face and the voxel is crossed an even number of times.  The origin is first moved along
// the line next to the voxel, which keeps the signed volumes accurate to about 1e-7 of the
// voxel size.  The crossing parameters, sorted, pair up into the voxel's intervals (two
// for a voxel that is slightly non-convex).
//
// Search.  Candidate voxels come from the pose's bin grid, walked by a 3D-DDA (Amanatides &
// Woo).  Within the current bin the next segment is the interval with the smallest
// (entry t, voxel id) after the last one returned whose entry t falls in the bin's t-range;
// a voxel listed in several bins is therefore taken in exactly one of them.
#pragma once
#include "nif_device.hpp"

namespace nif {

// Contraction of a*b+c into FMA is switched off for the traversal: the walk is inlined into
// several kernels (segment tracing, the fused query, the voxel proxy), which must take
// bit-identical decisions (entry parameters, crossing signs) for the same ray and voxel.
#pragma clang fp contract(off)

struct Ray {
    float3 o, d;
};

struct Trav {
    int32_t ix, iy, iz;
    float tmx, tmy, tmz;
    float tdx, tdy, tdz;  // t advance per bin along each axis
    int32_t ex, ey, ez;   // bin index at which the walk leaves the grid along each axis
    int32_t sx, sy, sz;   // step (+1 / -1)
    float t_lo;          // start of the current bin's t-range (-inf for the first bin)
    float last_a;        // key of the last returned segment
    int32_t last_cell;
    int32_t active;
};

__device__ __forceinline__ float3 f3sub(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float f3dot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 f3cross(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Local vertex m = bx + 2 by + 4 bz.  Canonical edges (lower local vertex first): 12 outer
// edges and the 6 face diagonals.  The 12 triangles, two per face, faces ordered x-low,
// x-high, y-low, y-high, z-low, z-high; a face (p00, p10, p11, p01) splits into
// (p00, p10, p11) and (p00, p11, p01).  Written out so every index is a compile-time constant.
struct CellHit {
    int n;               // intervals: 0, 1 or 2
    float a0, b0, a1, b1;
    int entry_face;      // face (0..5) of the first crossing
    int bad;             // odd or > 4 crossings (degenerate; reported as one interval)
};

__device__ __forceinline__ CellHit cell_intervals(const float4* __restrict__ V, int N, int cell, const Ray& R) {
    const int i = cell % N, j = (cell / N) % N, k = cell / (N * N);
    const int64_t n1 = N + 1;
    float3 v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        float4 q = V[(int64_t)(i + (m & 1)) + n1 * ((j + ((m >> 1) & 1)) + n1 * (k + (m >> 2)))];
        v[m] = make_float3(q.x, q.y, q.z);
    }
    const float dd = f3dot(R.d, R.d);
    const float tc = f3dot(f3sub(v[0], R.o), R.d) / dd;
    const float3 oc = make_float3(fmaf(tc, R.d.x, R.o.x), fmaf(tc, R.d.y, R.o.y), fmaf(tc, R.d.z, R.o.z));
    float3 p[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) p[m] = f3sub(v[m], oc);
    // edge signs for the canonical orientation; an exact zero counts as positive
#define NIF_E(a, b) (f3dot(R.d, f3cross(p[a], p[b])) >= 0.f)
    const bool e01 = NIF_E(0, 1), e23 = NIF_E(2, 3), e45 = NIF_E(4, 5), e67 = NIF_E(6, 7);
    const bool e02 = NIF_E(0, 2), e13 = NIF_E(1, 3), e46 = NIF_E(4, 6), e57 = NIF_E(5, 7);
    const bool e04 = NIF_E(0, 4), e15 = NIF_E(1, 5), e26 = NIF_E(2, 6), e37 = NIF_E(3, 7);
    const bool e06 = NIF_E(0, 6), e17 = NIF_E(1, 7), e05 = NIF_E(0, 5), e27 = NIF_E(2, 7);
    const bool e03 = NIF_E(0, 3), e47 = NIF_E(4, 7);
#undef NIF_E
    float t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f, tmax = -INFINITY;
    int cnt = 0, face0 = -1;
    // triangle (A, B, C) is crossed iff its three oriented edge signs agree
#define NIF_TRI(face, sab, sbc, sca, A, B, C)                                                   \
    if ((sab) == (sbc) && (sbc) == (sca)) {                                                     \
        const float3 n = f3cross(f3sub(p[B], p[A]), f3sub(p[C], p[A]));                         \
        const float den = f3dot(n, R.d);                                                        \
        float t = tc + (den != 0.f ? f3dot(n, p[A]) / den : 0.f);                               \
        /* insertion into the sorted prefix t0..t3 (more crossings only move tmax) */           \
        if (cnt == 0 || t < t0) face0 = (face);                                                 \
        if (cnt >= 1 && t < t0) { float x = t0; t0 = t; t = x; }                                \
        if (cnt >= 2 && t < t1) { float x = t1; t1 = t; t = x; }                                \
        if (cnt >= 3 && t < t2) { float x = t2; t2 = t; t = x; }                                \
        if (cnt >= 4 && t < t3) { float x = t3; t3 = t; t = x; }                                \
        if (cnt == 0) t0 = t; else if (cnt == 1) t1 = t; else if (cnt == 2) t2 = t; else if (cnt == 3) t3 = t; \
        tmax = fmaxf(tmax, t);                                                                  \
        ++cnt;                                                                                  \
    }
    NIF_TRI(0, e02, e26, !e06, 0, 2, 6) NIF_TRI(0, e06, !e46, !e04, 0, 6, 4)   // x-low
    NIF_TRI(1, e13, e37, !e17, 1, 3, 7) NIF_TRI(1, e17, !e57, !e15, 1, 7, 5)   // x-high
    NIF_TRI(2, e01, e15, !e05, 0, 1, 5) NIF_TRI(2, e05, !e45, !e04, 0, 5, 4)   // y-low
    NIF_TRI(3, e23, e37, !e27, 2, 3, 7) NIF_TRI(3, e27, !e67, !e26, 2, 7, 6)   // y-high
    NIF_TRI(4, e01, e13, !e03, 0, 1, 3) NIF_TRI(4, e03, !e23, !e02, 0, 3, 2)   // z-low
    NIF_TRI(5, e45, e57, !e47, 4, 5, 7) NIF_TRI(5, e47, !e67, !e46, 4, 7, 6)   // z-high
#undef NIF_TRI
    CellHit h;
    h.entry_face = face0;
    h.bad = 0;
    h.a1 = h.b1 = 0.f;
    if (cnt == 0) { h.n = 0; h.a0 = h.b0 = 0.f; }
    else if (cnt == 2) { h.n = 1; h.a0 = t0; h.b0 = t1; }
    else if (cnt == 4) { h.n = 2; h.a0 = t0; h.b0 = t1; h.a1 = t2; h.b1 = t3; }
    else { h.n = 1; h.a0 = t0; h.b0 = tmax; h.bad = 1; }
    return h;
}

// Enter the pose's bin grid.  Returns false if the ray misses it.
__device__ __forceinline__ void trav_init(const PoseDev& P, const Ray& R, Trav& T) {
    T.active = 0;
    T.last_a = -INFINITY;
    T.last_cell = -1;
    T.t_lo = -INFINITY;
    if (P.empty) return;
    float t0 = 0.f, t1 = INFINITY;
    bool miss = false;
    const float o[3] = {R.o.x, R.o.y, R.o.z}, d[3] = {R.d.x, R.d.y, R.d.z};
    const float plo[3] = {P.lo[0], P.lo[1], P.lo[2]}, pbs[3] = {P.bs[0], P.bs[1], P.bs[2]};
    const float pib[3] = {P.inv_bs[0], P.inv_bs[1], P.inv_bs[2]};
    const int pnb[3] = {P.nb[0], P.nb[1], P.nb[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = plo[a], hi = plo[a] + pnb[a] * pbs[a];
        if (d[a] == 0.f) {
            miss |= o[a] < lo || o[a] > hi;
        } else {
            const float ta = (lo - o[a]) / d[a], tb = (hi - o[a]) / d[a];
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        }
    }
    if (miss || t0 > t1) return;
    int idx[3];
    float tm[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float x = fmaf(t0, d[a], o[a]);
        const int c = (int)floorf((x - plo[a]) * pib[a]);
        idx[a] = min(max(c, 0), pnb[a] - 1);
        if (d[a] > 0.f) tm[a] = (plo[a] + (idx[a] + 1) * pbs[a] - o[a]) / d[a];
        else if (d[a] < 0.f) tm[a] = (plo[a] + idx[a] * pbs[a] - o[a]) / d[a];
        else tm[a] = INFINITY;
    }
    T.ix = idx[0]; T.iy = idx[1]; T.iz = idx[2];
    T.tmx = tm[0]; T.tmy = tm[1]; T.tmz = tm[2];
    T.tdx = d[0] != 0.f ? pbs[0] / fabsf(d[0]) : INFINITY;
    T.tdy = d[1] != 0.f ? pbs[1] / fabsf(d[1]) : INFINITY;
    T.tdz = d[2] != 0.f ? pbs[2] / fabsf(d[2]) : INFINITY;
    T.sx = d[0] > 0.f ? 1 : -1; T.sy = d[1] > 0.f ? 1 : -1; T.sz = d[2] > 0.f ? 1 : -1;
    T.ex = d[0] > 0.f ? pnb[0] : -1; T.ey = d[1] > 0.f ? pnb[1] : -1; T.ez = d[2] > 0.f ? pnb[2] : -1;
    T.active = 1;
}

struct Segment {
    int32_t cell;
    float a, b;
    int32_t face;
};

// Next occupied segment after T.last in front-to-back order.  Returns false when the ray
// has left the grid.  *bad counts degenerate voxel tests.
__device__ __forceinline__ bool next_segment(const PoseDev& P, const float4* __restrict__ V,
                                             const int32_t* __restrict__ bin_start,
                                             const int32_t* __restrict__ bin_cells, int N, const Ray& R,
                                             Trav& T, Segment& out, int* bad) {
    while (T.active) {
        // which face of the current bin the ray leaves through
        int ax = 0;
        float th = T.tmx;
        if (T.tmy < th) { ax = 1; th = T.tmy; }
        if (T.tmz < th) { ax = 2; th = T.tmz; }
        bool last;
        if (ax == 0) last = T.ix + T.sx == T.ex;
        else if (ax == 1) last = T.iy + T.sy == T.ey;
        else last = T.iz + T.sz == T.ez;
        last = last || !(th < INFINITY);
        const float t_hi = last ? INFINITY : th;
        const int64_t bin = (int64_t)T.ix + (int64_t)P.nb[0] * (T.iy + (int64_t)P.nb[1] * T.iz);
        const int32_t s0 = bin_start[P.bin_off + bin], s1 = bin_start[P.bin_off + bin + 1];
        float best_a = INFINITY, best_b = 0.f;
        int32_t best_c = 0x7fffffff, best_f = -1;
        for (int32_t e = s0; e < s1; ++e) {
            const int32_t c = bin_cells[P.ref_off + e];
            CellHit h = cell_intervals(V + P.vert_off, N, c, R);
            *bad += h.bad;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                if (q >= h.n) break;
                const float a = fmaxf(q == 0 ? h.a0 : h.a1, 0.f);
                const float b = q == 0 ? h.b0 : h.b1;
                if (!(b > a) || a < T.t_lo || !(a < t_hi)) continue;
                const bool after = a > T.last_a || (a == T.last_a && c > T.last_cell);
                const bool better = a < best_a || (a == best_a && c < best_c);
                if (after && better) { best_a = a; best_b = b; best_c = c; best_f = q == 0 ? h.entry_face : -1; }
            }
        }
        if (best_a < INFINITY) {
            T.last_a = best_a;
            T.last_cell = best_c;
            out.cell = best_c; out.a = best_a; out.b = best_b; out.face = best_f;
            return true;
        }
        if (last) { T.active = 0; return false; }
        T.t_lo = t_hi;
        if (ax == 0) { T.ix += T.sx; T.tmx += T.tdx; }
        else if (ax == 1) { T.iy += T.sy; T.tmy += T.tdy; }
        else { T.iz += T.sz; T.tmz += T.tdz; }
    }
    return false;
}

// Pose of ray r (rays are grouped by pose; offsets[0] = 0, offsets[n_poses] = n_rays).
__device__ __forceinline__ int find_pose(const int64_t* __restrict__ off, int n_poses, int64_t r) {
    int lo = 0, hi = n_poses - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

#pragma clang fp contract(fast)

}  // namespace nif
