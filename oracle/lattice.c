/*
 * Oracle (test infrastructure only): deformed voxel lattice and the ordered list of
 * occupied deformed voxels a ray crosses, in FP64.
 *
 * The paper voxelizes in rest space, deforms the voxels, and traces straight rays in
 * deformed space; because deformed voxels have non-uniform extents, the walk moves from
 * a voxel to the neighbour behind the face the ray exits through, starting from the
 * first voxel the ray meets (Methodology; "Voxel Traversal under Deformation").  The
 * entry and exit points of each occupied voxel are the endpoints of the ray segments
 * whose lengths are accumulated ("Segmented Ray Distance Accumulation").
 *
 * Reading used for the geometry of a deformed voxel (the paper gives none): the lattice
 * vertices V_ijk = D(i/N, j/N, k/N); each face is the quad of its four deformed corners,
 * split along its main diagonal into two triangles, so neighbouring voxels share exactly
 * the same face and the deformed lattice is watertight.  For a face whose corners are
 * a, a+e1, a+e1+e2, a+e2 (e1 the lower of the two in-face axes) the triangles are
 * (a, a+e1, a+e1+e2) and (a, a+e1+e2, a+e2).
 *
 * The hit list of a ray o + t d (t over the whole line) is defined by its crossings with
 * lattice faces, sorted by t: starting outside, each crossing moves to the voxel on the
 * other side of the face.  Each visit gives an interval [t_in, t_out]; intervals are
 * clipped to t >= 0 and the occupied voxels with t_out > t_in are kept, in order.
 *
 * Two ways to compute it are provided and must agree: `brute` tests every face of the
 * lattice and sorts; the walk follows the paper (exit face of the current voxel; the
 * boundary faces when outside, which also covers re-entry into a non-convex lattice).
 *
 * Rays for which FP rounding could legitimately change the list are flagged "grazing"
 * (threshold 1e-6 in deformed-space distance) and are compared separately:
 *   1  a crossing of a face next to an occupied voxel within 1e-6 of one of the quad's
 *      four outer edges (the diagonal does not matter: both triangles belong to the face);
 *   2  |n . d| < 1e-6 at such a crossing (n the unit normal of the crossed triangle);
 *   4  the origin within 1e-6 of a face of the voxel that contains it;
 *   8  the line within 1e-6 of an edge of an occupied voxel;
 *   16 an inconsistent walk (a crossing that is not a face of the current voxel).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define GRAZE 1e-6

typedef struct { double t; int32_t face, lo, hi, tri; } xing;

static int64_t vid(int32_t N, int i, int j, int k) {
    return i + (int64_t)(N + 1) * (j + (int64_t)(N + 1) * k);
}

void orc_lattice_vertices(int kind, double s, int32_t N, double* V) {
    for (int k = 0; k <= N; ++k)
        for (int j = 0; j <= N; ++j)
            for (int i = 0; i <= N; ++i) {
                double p[3] = {(double)i / N, (double)j / N, (double)k / N};
                orc_deform(kind, s, p, V + 3 * vid(N, i, j, k));
            }
}

/* Face (a, w, u, v): normal axis a, lattice coordinate w in [0, N] along a, and the
   lower corner (u, v) in [0, N)^2 along the two in-face axes e1 < e2. */
static void face_axes(int a, int* e1, int* e2) {
    *e1 = (a == 0) ? 1 : 0;
    *e2 = (a == 2) ? 1 : 2;
}

static int32_t face_id(int32_t N, int a, int w, int u, int v) {
    return ((a * (N + 1) + w) * N + u) * N + v;
}

static void face_decode(int32_t N, int32_t f, int* a, int* w, int* u, int* v) {
    *v = f % N; f /= N;
    *u = f % N; f /= N;
    *w = f % (N + 1); *a = f / (N + 1);
}

static int32_t cell_id(int32_t N, const int c[3]) {
    return c[0] + N * (c[1] + N * c[2]);
}

/* The two cells on either side of a face (-1 outside the lattice). */
static void face_cells(int32_t N, int a, int w, int u, int v, int32_t* lo, int32_t* hi) {
    int e1, e2, c[3];
    face_axes(a, &e1, &e2);
    c[e1] = u; c[e2] = v;
    c[a] = w - 1; *lo = (w >= 1) ? cell_id(N, c) : -1;
    c[a] = w;     *hi = (w <= N - 1) ? cell_id(N, c) : -1;
}

static void face_quad(int32_t N, const double* V, int a, int w, int u, int v, const double* q[4]) {
    int e1, e2, c[3];
    face_axes(a, &e1, &e2);
    c[a] = w;
    c[e1] = u;     c[e2] = v;     q[0] = V + 3 * vid(N, c[0], c[1], c[2]);
    c[e1] = u + 1; c[e2] = v;     q[1] = V + 3 * vid(N, c[0], c[1], c[2]);
    c[e1] = u + 1; c[e2] = v + 1; q[2] = V + 3 * vid(N, c[0], c[1], c[2]);
    c[e1] = u;     c[e2] = v + 1; q[3] = V + 3 * vid(N, c[0], c[1], c[2]);
}

static void sub3(const double* a, const double* b, double* r) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

/* Moller-Trumbore line/triangle test, no culling, inclusive edges.  Returns 1 and the
   line parameter t if the line o + t d crosses triangle (A, B, C). */
static int line_tri(const double* o, const double* d, const double* A, const double* B,
                    const double* C, double* t) {
    double e1[3], e2[3], p[3], s[3], q[3];
    sub3(B, A, e1); sub3(C, A, e2);
    cross3(d, e2, p);
    double det = dot3(e1, p);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    sub3(o, A, s);
    double u = dot3(s, p) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    cross3(s, e1, q);
    double v = dot3(d, q) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    *t = dot3(e2, q) * inv;
    return 1;
}

/* Crossings of the line with one face: 0, 1 or 2 (one per triangle). */
static int face_cross(int32_t N, const double* V, int32_t f, const double* o, const double* d,
                      xing* out) {
    int a, w, u, v, n = 0;
    face_decode(N, f, &a, &w, &u, &v);
    const double* q[4];
    face_quad(N, V, a, w, u, v, q);
    int32_t lo, hi;
    face_cells(N, a, w, u, v, &lo, &hi);
    double t;
    if (line_tri(o, d, q[0], q[1], q[2], &t)) { out[n].t = t; out[n].face = f; out[n].lo = lo; out[n].hi = hi; out[n].tri = 0; ++n; }
    if (line_tri(o, d, q[0], q[2], q[3], &t)) { out[n].t = t; out[n].face = f; out[n].lo = lo; out[n].hi = hi; out[n].tri = 1; ++n; }
    return n;
}

static double point_segment_dist(const double* X, const double* A, const double* B) {
    double e[3], w[3];
    sub3(B, A, e); sub3(X, A, w);
    double c = dot3(e, e);
    double s = c > 0.0 ? dot3(w, e) / c : 0.0;
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    double r[3] = {A[0] + s * e[0] - X[0], A[1] + s * e[1] - X[1], A[2] + s * e[2] - X[2]};
    return sqrt(dot3(r, r));
}

/* Distance between the infinite line o + t d and the segment [A, B]: the squared distance
   from A + s(B-A) to the line is a convex quadratic in s; minimise it and clamp s to [0,1]. */
static double line_segment_dist(const double* o, const double* d, const double* A, const double* B) {
    double e[3], w0[3];
    sub3(B, A, e); sub3(A, o, w0);
    double a = dot3(d, d), b = dot3(d, e), c = dot3(e, e);
    double dd = dot3(d, w0), ee = dot3(e, w0);
    double den = a * c - b * b;
    double s = den > 1e-300 ? (b * dd - a * ee) / den : 0.0;   /* parallel: any s */
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    double w[3] = {w0[0] + s * e[0], w0[1] + s * e[1], w0[2] + s * e[2]};
    double t = dot3(w, d) / a;
    double r[3] = {w[0] - t * d[0], w[1] - t * d[1], w[2] - t * d[2]};
    return sqrt(dot3(r, r));
}

/* Closest distance from a point to a triangle (region tests on barycentric coordinates). */
static double point_tri_dist(const double* p, const double* a, const double* b, const double* c) {
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    sub3(b, a, ab); sub3(c, a, ac); sub3(p, a, ap);
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    double r[3];
    if (d1 <= 0 && d2 <= 0) { sub3(p, a, r); return sqrt(dot3(r, r)); }
    sub3(p, b, bp);
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0 && d4 <= d3) { sub3(p, b, r); return sqrt(dot3(r, r)); }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0 && d1 >= 0 && d3 <= 0) return point_segment_dist(p, a, b);
    sub3(p, c, cp);
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0 && d5 <= d6) { sub3(p, c, r); return sqrt(dot3(r, r)); }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0 && d2 >= 0 && d6 <= 0) return point_segment_dist(p, a, c);
    double va = d3 * d6 - d5 * d4;
    if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) return point_segment_dist(p, b, c);
    double den = 1.0 / (va + vb + vc);
    double v = vb * den, w = vc * den;
    double q[3] = {a[0] + ab[0] * v + ac[0] * w, a[1] + ab[1] * v + ac[1] * w, a[2] + ab[2] * v + ac[2] * w};
    sub3(p, q, r);
    return sqrt(dot3(r, r));
}

/* Grazing flags 1 and 2 of one crossing (only faces next to an occupied voxel matter). */
static int32_t crossing_flags(int32_t N, const uint8_t* occ, const double* V, const xing* x,
                              const double* o, const double* d) {
    int occ_adj = (x->lo >= 0 && occ[x->lo]) || (x->hi >= 0 && occ[x->hi]);
    if (!occ_adj) return 0;
    int a, w, u, v;
    face_decode(N, x->face, &a, &w, &u, &v);
    const double* q[4];
    face_quad(N, V, a, w, u, v, q);
    double X[3] = {o[0] + x->t * d[0], o[1] + x->t * d[1], o[2] + x->t * d[2]};
    int32_t fl = 0;
    for (int e = 0; e < 4; ++e)
        if (point_segment_dist(X, q[e], q[(e + 1) & 3]) < GRAZE) fl |= 1;
    const double* A = q[0];
    const double* B = x->tri == 0 ? q[1] : q[2];
    const double* C = x->tri == 0 ? q[2] : q[3];
    double e1[3], e2[3], n[3];
    sub3(B, A, e1); sub3(C, A, e2); cross3(e1, e2, n);
    double nl = sqrt(dot3(n, n));
    if (nl > 0.0 && fabs(dot3(n, d)) / nl < GRAZE) fl |= 2;
    return fl;
}

static int cmp_xing(const void* pa, const void* pb) {
    const xing* a = (const xing*)pa;
    const xing* b = (const xing*)pb;
    if (a->t < b->t) return -1;
    if (a->t > b->t) return 1;
    return (a->face > b->face) - (a->face < b->face);
}

static int same_point(double t0, double t1) {
    double m = fabs(t0) > 1.0 ? fabs(t0) : 1.0;
    return fabs(t1 - t0) <= 1e-12 * m;
}

/* All face crossings of the line, in order, by exhaustive testing of every face. */
static int brute_crossings(int32_t N, const double* V, const double* o, const double* d,
                           xing** out) {
    int64_t nfaces = 3LL * (N + 1) * N * N;
    int cap = 64, n = 0;
    xing* xs = (xing*)malloc(sizeof(xing) * cap);
    for (int64_t f = 0; f < nfaces; ++f) {
        xing tmp[2];
        int k = face_cross(N, V, (int32_t)f, o, d, tmp);
        for (int i = 0; i < k; ++i) {
            if (n == cap) { cap *= 2; xs = (xing*)realloc(xs, sizeof(xing) * cap); }
            xs[n++] = tmp[i];
        }
    }
    qsort(xs, n, sizeof(xing), cmp_xing);
    /* both triangles of a quad report a crossing on their shared diagonal: merge */
    int m = 0;
    for (int i = 0; i < n; ++i) {
        if (m > 0 && xs[m - 1].face == xs[i].face && same_point(xs[m - 1].t, xs[i].t)) continue;
        xs[m++] = xs[i];
    }
    *out = xs;
    return m;
}

/* All face crossings of the line, in order, by the exit-face walk. */
static int walk_crossings(int32_t N, const double* V, const double* o, const double* d,
                          xing** out, int32_t* flags) {
    int cap = 64, n = 0;
    xing* xs = (xing*)malloc(sizeof(xing) * cap);
    int32_t cur = -1, fin = -1;
    double tcur = -INFINITY;
    for (;;) {
        xing best;
        best.face = -1; best.t = INFINITY;
        xing tmp[2];
        if (cur < 0) {
            for (int a = 0; a < 3; ++a)
                for (int side = 0; side < 2; ++side) {
                    int w = side ? N : 0;
                    for (int u = 0; u < N; ++u)
                        for (int v = 0; v < N; ++v) {
                            int32_t f = face_id(N, a, w, u, v);
                            int k = face_cross(N, V, f, o, d, tmp);
                            for (int i = 0; i < k; ++i) {
                                if (!(tmp[i].t > tcur)) continue;
                                if (f == fin && same_point(tcur, tmp[i].t)) continue;
                                if (tmp[i].t < best.t) best = tmp[i];
                            }
                        }
                }
            if (best.face < 0) break;                 /* no more boundary crossings */
        } else {
            int c[3] = {cur % N, (cur / N) % N, cur / (N * N)};
            for (int a = 0; a < 3; ++a) {
                int e1, e2;
                face_axes(a, &e1, &e2);
                for (int side = 0; side < 2; ++side) {
                    int32_t f = face_id(N, a, c[a] + side, c[e1], c[e2]);
                    int k = face_cross(N, V, f, o, d, tmp);
                    for (int i = 0; i < k; ++i) {
                        if (!(tmp[i].t > tcur)) continue;
                        if (f == fin && same_point(tcur, tmp[i].t)) continue;
                        if (tmp[i].t < best.t) best = tmp[i];
                    }
                }
            }
            if (best.face < 0) { *flags |= 16; break; }   /* a closed voxel must be left */
        }
        if (n == cap) { cap *= 2; xs = (xing*)realloc(xs, sizeof(xing) * cap); }
        xs[n++] = best;
        if (cur == best.lo) cur = best.hi;
        else if (cur == best.hi) cur = best.lo;
        else { *flags |= 16; break; }
        tcur = best.t;
        fin = best.face;
    }
    *out = xs;
    return n;
}

/* |cos| of the angle between the line and the normal of the crossed triangle. */
static double crossing_cos(int32_t N, const double* V, const xing* x, const double* d) {
    int a, w, u, v;
    face_decode(N, x->face, &a, &w, &u, &v);
    const double* q[4];
    face_quad(N, V, a, w, u, v, q);
    const double* A = q[0];
    const double* B = x->tri == 0 ? q[1] : q[2];
    const double* C = x->tri == 0 ? q[2] : q[3];
    double e1[3], e2[3], n[3];
    sub3(B, A, e1); sub3(C, A, e2); cross3(e1, e2, n);
    double den = sqrt(dot3(n, n) * dot3(d, d));
    return den > 0.0 ? fabs(dot3(n, d)) / den : 0.0;
}

int32_t orc_hitlist(int32_t N, const uint8_t* occ, const double* V, const double o[3], const double d[3],
                    int32_t brute, int32_t max_out, int32_t* cell, double* tin, double* tout,
                    int32_t* flags, double* cin, double* cout) {
    xing* xs = NULL;
    int32_t fl = 0;
    int n = brute ? brute_crossings(N, V, o, d, &xs) : walk_crossings(N, V, o, d, &xs, &fl);
    int32_t cur = -1, start_cell = -1, count = 0;
    double tprev = -INFINITY, cprev = 1.0;
    for (int i = 0; i < n; ++i) {
        const xing* x = &xs[i];
        if (flags) fl |= crossing_flags(N, occ, V, x, o, d);
        int32_t next;
        if (cur == x->lo) next = x->hi;
        else if (cur == x->hi) next = x->lo;
        else { fl |= 16; break; }
        if (cur >= 0) {
            double a = tprev > 0.0 ? tprev : 0.0, b = x->t;
            if (tprev <= 0.0 && b > 0.0) start_cell = cur;
            if (b > a && occ[cur]) {
                if (count < max_out) {
                    cell[count] = cur; tin[count] = a; tout[count] = b;
                    if (cin) cin[count] = tprev > 0.0 ? cprev : 1.0;   /* clipped start: no crossing */
                    if (cout) cout[count] = crossing_cos(N, V, x, d);
                }
                ++count;
            }
        }
        cur = next;
        tprev = x->t;
        if (cin) cprev = crossing_cos(N, V, x, d);
    }
    if (cur != -1) fl |= 16;
    free(xs);
    if (!flags) return count;

    /* flag 4: origin close to a face of the voxel that contains it */
    if (start_cell >= 0) {
        int c[3] = {start_cell % N, (start_cell / N) % N, start_cell / (N * N)};
        for (int a = 0; a < 3; ++a) {
            int e1, e2;
            face_axes(a, &e1, &e2);
            for (int side = 0; side < 2; ++side) {
                const double* q[4];
                face_quad(N, V, a, c[a] + side, c[e1], c[e2], q);
                if (point_tri_dist(o, q[0], q[1], q[2]) < GRAZE || point_tri_dist(o, q[0], q[2], q[3]) < GRAZE)
                    fl |= 4;
            }
        }
    }
    /* flag 8: line close to an edge of an occupied voxel */
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                if (!occ[i + N * (j + N * k)]) continue;
                const double* cv[8];
                double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
                for (int m = 0; m < 8; ++m) {
                    cv[m] = V + 3 * vid(N, i + (m & 1), j + ((m >> 1) & 1), k + (m >> 2));
                    for (int c = 0; c < 3; ++c) {
                        if (cv[m][c] < lo[c]) lo[c] = cv[m][c];
                        if (cv[m][c] > hi[c]) hi[c] = cv[m][c];
                    }
                }
                /* skip voxels whose padded box the line misses (slab test) */
                double t0 = -INFINITY, t1 = INFINITY;
                int miss = 0;
                for (int c = 0; c < 3 && !miss; ++c) {
                    double l = lo[c] - 2 * GRAZE, h = hi[c] + 2 * GRAZE;
                    if (d[c] == 0.0) { if (o[c] < l || o[c] > h) miss = 1; continue; }
                    double ta = (l - o[c]) / d[c], tb = (h - o[c]) / d[c];
                    if (ta > tb) { double s = ta; ta = tb; tb = s; }
                    if (ta > t0) t0 = ta;
                    if (tb < t1) t1 = tb;
                    if (t0 > t1) miss = 1;
                }
                if (miss) continue;
                for (int m = 0; m < 8; ++m)
                    for (int ax = 0; ax < 3; ++ax) {
                        if (m & (1 << ax)) continue;
                        if (line_segment_dist(o, d, cv[m], cv[m | (1 << ax)]) < GRAZE) fl |= 8;
                    }
            }
    *flags = fl;
    return count;
}
