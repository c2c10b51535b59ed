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

struct Ray {
    float3 o, d;
};

struct Trav {
    int32_t ix, iy, iz;
    float tmx, tmy, tmz;
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

// Canonical edges (lower local vertex first); local vertex m = bx + 2 by + 4 bz.
__device__ constexpr int kEdgeA[18] = {0, 2, 4, 6, 0, 1, 4, 5, 0, 1, 2, 3, 0, 1, 0, 2, 0, 4};
__device__ constexpr int kEdgeB[18] = {1, 3, 5, 7, 2, 3, 6, 7, 4, 5, 6, 7, 6, 7, 5, 7, 3, 7};
// 12 triangles, two per face, faces ordered x-low, x-high, y-low, y-high, z-low, z-high;
// each face (p00, p10, p11, p01) splits into (p00, p10, p11) and (p00, p11, p01).
__device__ constexpr int kTriV[12][3] = {{0, 2, 6}, {0, 6, 4}, {1, 3, 7}, {1, 7, 5}, {0, 1, 5}, {0, 5, 4},
                                         {2, 3, 7}, {2, 7, 6}, {0, 1, 3}, {0, 3, 2}, {4, 5, 7}, {4, 7, 6}};
// edge index and orientation (1 = reversed) of the triangle edges A->B, B->C, C->A
__device__ constexpr int kTriE[12][3] = {{4, 10, 12}, {12, 6, 8}, {5, 11, 13}, {13, 7, 9}, {0, 9, 14}, {14, 2, 8},
                                         {1, 11, 15}, {15, 3, 10}, {0, 5, 16}, {16, 1, 4}, {2, 7, 17}, {17, 3, 6}};
__device__ constexpr int kTriR[12][3] = {{0, 0, 1}, {0, 1, 1}, {0, 0, 1}, {0, 1, 1}, {0, 0, 1}, {0, 1, 1},
                                         {0, 0, 1}, {0, 1, 1}, {0, 0, 1}, {0, 1, 1}, {0, 0, 1}, {0, 1, 1}};

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
    bool s[18];
#pragma unroll
    for (int e = 0; e < 18; ++e) s[e] = f3dot(R.d, f3cross(p[kEdgeA[e]], p[kEdgeB[e]])) >= 0.f;
    float t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f, tmax = -INFINITY;
    int cnt = 0, face0 = -1;
#pragma unroll
    for (int tr = 0; tr < 12; ++tr) {
        bool s0 = s[kTriE[tr][0]] != (bool)kTriR[tr][0];
        bool s1 = s[kTriE[tr][1]] != (bool)kTriR[tr][1];
        bool s2 = s[kTriE[tr][2]] != (bool)kTriR[tr][2];
        if (s0 == s1 && s1 == s2) {
            const float3 A = p[kTriV[tr][0]], B = p[kTriV[tr][1]], C = p[kTriV[tr][2]];
            const float3 n = f3cross(f3sub(B, A), f3sub(C, A));
            const float den = f3dot(n, R.d);
            float t = tc + (den != 0.f ? f3dot(n, A) / den : 0.f);
            // insertion into the sorted prefix t0..t3 (later crossings beyond 4 only move tmax)
            if (cnt == 0 || t < t0) face0 = tr >> 1;
            if (cnt >= 1 && t < t0) { float x = t0; t0 = t; t = x; }
            if (cnt >= 2 && t < t1) { float x = t1; t1 = t; t = x; }
            if (cnt >= 3 && t < t2) { float x = t2; t2 = t; t = x; }
            if (cnt >= 4 && t < t3) { float x = t3; t3 = t; t = x; }
            if (cnt == 0) t0 = t; else if (cnt == 1) t1 = t; else if (cnt == 2) t2 = t; else if (cnt == 3) t3 = t;
            tmax = fmaxf(tmax, t);
            ++cnt;
        }
    }
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
    const float o[3] = {R.o.x, R.o.y, R.o.z}, d[3] = {R.d.x, R.d.y, R.d.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = P.lo[a], hi = P.lo[a] + P.nb[a] * P.bs[a];
        if (d[a] == 0.f) {
            if (o[a] < lo || o[a] > hi) return;
        } else {
            float ta = (lo - o[a]) / d[a], tb = (hi - o[a]) / d[a];
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        }
    }
    if (t0 > t1) return;
    int idx[3];
    float tm[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float x = fmaf(t0, d[a], o[a]);
        int c = (int)floorf((x - P.lo[a]) * P.inv_bs[a]);
        idx[a] = min(max(c, 0), P.nb[a] - 1);
        if (d[a] > 0.f) tm[a] = (P.lo[a] + (idx[a] + 1) * P.bs[a] - o[a]) / d[a];
        else if (d[a] < 0.f) tm[a] = (P.lo[a] + idx[a] * P.bs[a] - o[a]) / d[a];
        else tm[a] = INFINITY;
    }
    T.ix = idx[0]; T.iy = idx[1]; T.iz = idx[2];
    T.tmx = tm[0]; T.tmy = tm[1]; T.tmz = tm[2];
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
    const float d[3] = {R.d.x, R.d.y, R.d.z};
    while (T.active) {
        // which face of the current bin the ray leaves through
        int ax = 0;
        float th = T.tmx;
        if (T.tmy < th) { ax = 1; th = T.tmy; }
        if (T.tmz < th) { ax = 2; th = T.tmz; }
        const int cur = ax == 0 ? T.ix : (ax == 1 ? T.iy : T.iz);
        const int stp = d[ax] > 0.f ? 1 : -1;
        const bool last = (cur + stp < 0) || (cur + stp >= P.nb[ax]) || !(th < INFINITY);
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
        const float bsd = P.bs[ax] / fabsf(d[ax]);
        if (ax == 0) { T.ix += stp; T.tmx += bsd; }
        else if (ax == 1) { T.iy += stp; T.tmy += bsd; }
        else { T.iz += stp; T.tmz += bsd; }
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

}  // namespace nif
