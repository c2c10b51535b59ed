/*
 * Oracle (test infrastructure only): synthetic implicit scenes, rest-space voxelization
 * and ground-truth labels, in FP64.
 *
 * The paper voxelizes the geometry in rest space (Methodology) and labels each
 * locally-linearized rest-space ray segment by intersecting it with the rest geometry,
 * producing hit/occlusion, distance, normal, albedo and material (Methodology, the
 * paragraph on the local linear approximation).  Its meshes are not available; the
 * scenes here are implicit surfaces f(p) with f < 0 inside:
 *   torus  : params [cx,cy,cz,R,r], f = (sqrt((x-cx)^2+(y-cy)^2) - R)^2 + (z-cz)^2 - r^2,
 *            albedo_c = 0.5 + 0.4 sin(2 pi (2 p_c + c/3)), material = [x >= 0.5];
 *   spheres: params [n, (cx,cy,cz,r, ar,ag,ab, mat) x n], f = min_i |p-c_i| - r_i,
 *            attributes of the minimizing sphere;
 *   blobs  : params [n, (mx,my,mz,sigma, cr,cg,cb, mat) x n],
 *            f = 0.5 - sum_i exp(-|p-m_i|^2 / (2 sigma_i^2)), albedo = contribution-weighted
 *            mean colour, material = that of the largest contribution.
 */
#include <math.h>
#include "oracle.h"

#define SPH_STRIDE 8

double orc_scene_f(int kind, const double* sp, const double p[3]) {
    if (kind == ORC_SCENE_TORUS) {
        double dx = p[0] - sp[0], dy = p[1] - sp[1], dz = p[2] - sp[2];
        double q = sqrt(dx * dx + dy * dy) - sp[3];
        return q * q + dz * dz - sp[4] * sp[4];
    }
    if (kind == ORC_SCENE_SPHERES) {
        int n = (int)sp[0];
        double best = INFINITY;
        for (int i = 0; i < n; ++i) {
            const double* c = sp + 1 + SPH_STRIDE * i;
            double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
            double v = sqrt(dx * dx + dy * dy + dz * dz) - c[3];
            if (v < best) best = v;
        }
        return best;
    }
    /* blobs */
    int n = (int)sp[0];
    double g = 0.0;
    for (int i = 0; i < n; ++i) {
        const double* b = sp + 1 + SPH_STRIDE * i;
        double dx = p[0] - b[0], dy = p[1] - b[1], dz = p[2] - b[2];
        g += exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * b[3] * b[3]));
    }
    return 0.5 - g;
}

void orc_scene_grad(int kind, const double* sp, const double p[3], double g[3]) {
    if (kind == ORC_SCENE_TORUS) {
        double dx = p[0] - sp[0], dy = p[1] - sp[1], dz = p[2] - sp[2];
        double rho = sqrt(dx * dx + dy * dy);
        double q = rho - sp[3];
        double k = rho > 0.0 ? 2.0 * q / rho : 0.0;
        g[0] = k * dx; g[1] = k * dy; g[2] = 2.0 * dz;
        return;
    }
    if (kind == ORC_SCENE_SPHERES) {
        int n = (int)sp[0], arg = 0;
        double best = INFINITY;
        for (int i = 0; i < n; ++i) {
            const double* c = sp + 1 + SPH_STRIDE * i;
            double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
            double v = sqrt(dx * dx + dy * dy + dz * dz) - c[3];
            if (v < best) { best = v; arg = i; }
        }
        const double* c = sp + 1 + SPH_STRIDE * arg;
        double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r == 0.0) { g[0] = 0; g[1] = 0; g[2] = 1; return; }
        g[0] = dx / r; g[1] = dy / r; g[2] = dz / r;
        return;
    }
    int n = (int)sp[0];
    g[0] = g[1] = g[2] = 0.0;
    for (int i = 0; i < n; ++i) {
        const double* b = sp + 1 + SPH_STRIDE * i;
        double dx = p[0] - b[0], dy = p[1] - b[1], dz = p[2] - b[2];
        double s2 = b[3] * b[3];
        double e = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s2));
        /* d f / d p = - d g / d p = sum e * (p - m) / sigma^2 */
        g[0] += e * dx / s2; g[1] += e * dy / s2; g[2] += e * dz / s2;
    }
}

void orc_scene_attr(int kind, const double* sp, const double p[3], double albedo[3], int32_t* material) {
    if (kind == ORC_SCENE_TORUS) {
        for (int c = 0; c < 3; ++c)
            albedo[c] = 0.5 + 0.4 * sin(2.0 * M_PI * (2.0 * p[c] + c / 3.0));
        *material = p[0] >= 0.5 ? 1 : 0;
        return;
    }
    if (kind == ORC_SCENE_SPHERES) {
        int n = (int)sp[0], arg = 0;
        double best = INFINITY;
        for (int i = 0; i < n; ++i) {
            const double* c = sp + 1 + SPH_STRIDE * i;
            double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
            double v = sqrt(dx * dx + dy * dy + dz * dz) - c[3];
            if (v < best) { best = v; arg = i; }
        }
        const double* c = sp + 1 + SPH_STRIDE * arg;
        albedo[0] = c[4]; albedo[1] = c[5]; albedo[2] = c[6];
        *material = (int32_t)c[7];
        return;
    }
    int n = (int)sp[0], arg = 0;
    double wsum = 0.0, wbest = -1.0;
    albedo[0] = albedo[1] = albedo[2] = 0.0;
    for (int i = 0; i < n; ++i) {
        const double* b = sp + 1 + SPH_STRIDE * i;
        double dx = p[0] - b[0], dy = p[1] - b[1], dz = p[2] - b[2];
        double e = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * b[3] * b[3]));
        wsum += e;
        albedo[0] += e * b[4]; albedo[1] += e * b[5]; albedo[2] += e * b[6];
        if (e > wbest) { wbest = e; arg = i; }
    }
    if (wsum > 0.0) { albedo[0] /= wsum; albedo[1] /= wsum; albedo[2] /= wsum; }
    *material = (int32_t)sp[1 + SPH_STRIDE * arg + 7];
}

/* Cell (i,j,k) of the N^3 grid over [0,1]^3 is occupied iff f, sampled on the 5^3
   sub-lattice of the closed cell (corners included), takes both signs (min <= 0 <= max).
   Layout: occ[i + N*(j + N*k)]. */
void orc_voxelize(int kind, const double* sp, int32_t N, uint8_t* occ) {
    const int sub = 4;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                double lo = INFINITY, hi = -INFINITY;
                for (int c = 0; c <= sub; ++c)
                    for (int b = 0; b <= sub; ++b)
                        for (int a = 0; a <= sub; ++a) {
                            double p[3] = {(i + (double)a / sub) / N, (j + (double)b / sub) / N,
                                           (k + (double)c / sub) / N};
                            double v = orc_scene_f(kind, sp, p);
                            if (v < lo) lo = v;
                            if (v > hi) hi = v;
                        }
                occ[i + (int64_t)N * (j + (int64_t)N * k)] = (lo <= 0.0 && hi >= 0.0) ? 1 : 0;
            }
}

/* First point on the rest segment x(tau) = x0 + tau*u, tau in [0, len], where f <= 0.
   Spheres use the closed-form quadratic unless force_march is set; everything else
   takes 256 uniform sign steps and bisects the first bracket down to 1e-13. */
static int first_inside(int kind, const double* sp, int force_march, const double x0[3],
                        const double u[3], double len, double* tau) {
    double f0 = orc_scene_f(kind, sp, x0);
    if (f0 <= 0.0) { *tau = 0.0; return 1; }
    if (len <= 0.0) return 0;
    if (kind == ORC_SCENE_SPHERES && !force_march) {
        int n = (int)sp[0], found = 0;
        double best = INFINITY;
        for (int i = 0; i < n; ++i) {
            const double* c = sp + 1 + SPH_STRIDE * i;
            double w[3] = {x0[0] - c[0], x0[1] - c[1], x0[2] - c[2]};
            double b = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
            double cc = w[0] * w[0] + w[1] * w[1] + w[2] * w[2] - c[3] * c[3];
            double disc = b * b - cc;
            if (disc < 0.0) continue;
            double r = -b - sqrt(disc);   /* entering root; x0 is outside every sphere */
            if (r >= 0.0 && r <= len && r < best) { best = r; found = 1; }
        }
        if (found) *tau = best;
        return found;
    }
    const int steps = 256;
    double prev = 0.0;
    for (int s = 1; s <= steps; ++s) {
        double t = len * s / steps;
        double p[3] = {x0[0] + t * u[0], x0[1] + t * u[1], x0[2] + t * u[2]};
        if (orc_scene_f(kind, sp, p) <= 0.0) {
            double a = prev, b = t;           /* f(a) > 0 >= f(b) */
            while (b - a > 1e-13) {
                double m = 0.5 * (a + b);
                double q[3] = {x0[0] + m * u[0], x0[1] + m * u[1], x0[2] + m * u[2]};
                if (orc_scene_f(kind, sp, q) <= 0.0) b = m; else a = m;
            }
            *tau = b;
            return 1;
        }
        prev = t;
    }
    return 0;
}

void orc_label(int kind, const double* sp, int force_march, const double x0[3], const double x1[3],
               uint8_t* hit, double* t, double n[3], double a[3], int32_t* m) {
    double e[3] = {x1[0] - x0[0], x1[1] - x0[1], x1[2] - x0[2]};
    double len = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    double u[3] = {0.0, 0.0, 0.0};
    if (len > 0.0) { u[0] = e[0] / len; u[1] = e[1] / len; u[2] = e[2] / len; }
    double tau = 0.0;
    *hit = (uint8_t)first_inside(kind, sp, force_march, x0, u, len, &tau);
    n[0] = n[1] = n[2] = 0.0; a[0] = a[1] = a[2] = 0.0; *m = 0; *t = 0.0;
    if (!*hit) return;
    *t = tau;
    double p[3] = {x0[0] + tau * u[0], x0[1] + tau * u[1], x0[2] + tau * u[2]};
    double g[3];
    orc_scene_grad(kind, sp, p, g);
    double gl = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (gl > 0.0) { n[0] = g[0] / gl; n[1] = g[1] / gl; n[2] = g[2] / gl; }
    orc_scene_attr(kind, sp, p, a, m);
}
