/*
 * Oracle (test infrastructure only): parameterized deformations of the rest space and
 * their analytic inverses, in FP64.
 *
 * The paper maps every deformed-space sample back to the canonical rest space through
 * the inverse of a user-parameterized deformation (Methodology, opening paragraphs; the
 * twist warp of Figure 2).  It gives no formulas; these are the classic global
 * deformations (twist, bend, taper) with the pivot at the cube centre and one strength
 * s in [0, 1] per pose:
 *   twist: rotation about the z axis through the centre by theta = 0.6 s z radians;
 *   bend : circular bend in the x-z plane, curvature kappa = s / 1.5 (radius 1.5 at s=1);
 *   taper: x,y scaled about the centre by sigma(z) = 1 - 0.5 s z;
 *   twist-bend: the twist followed by the bend, both at strength s (a composed pose: the
 *   method only needs D and its inverse, so compositions are poses like any other).
 *
 * Deformed-space normals (the network predicts rest-space normals; a renderer working in
 * deformed space needs the normal of the deformed surface): a normal transforms with the
 * inverse transpose of the Jacobian J = dD/dp at the rest point.  J is taken by central
 * differences of D (step 1e-6, error ~1e-10), inverted with the adjugate formula.
 */
#include <math.h>
#include "oracle.h"

#define CX 0.5
#define CY 0.5
#define CZ 0.5

void orc_deform(int kind, double s, const double p[3], double q[3]) {
    if (kind == ORC_TWIST_BEND) {
        double t[3];
        orc_deform(ORC_TWIST, s, p, t);
        orc_deform(ORC_BEND, s, t, q);
        return;
    }
    q[0] = p[0]; q[1] = p[1]; q[2] = p[2];
    if (kind == ORC_TWIST) {
        double th = 0.6 * s * p[2];
        double x = p[0] - CX, y = p[1] - CY;
        q[0] = CX + cos(th) * x - sin(th) * y;
        q[1] = CY + sin(th) * x + cos(th) * y;
    } else if (kind == ORC_BEND) {
        double k = s / 1.5;
        if (k == 0.0) return;
        double u = p[0] - CX, ph = k * (p[2] - CZ);
        /* the rest point at signed distance u from the centre line lies on a circle of
           radius 1/k - u about (CX + 1/k, CZ); ph is its angle */
        q[0] = CX + 1.0 / k - (1.0 / k - u) * cos(ph);
        q[2] = CZ + (1.0 / k - u) * sin(ph);
    } else if (kind == ORC_TAPER) {
        double sg = 1.0 - 0.5 * s * p[2];
        q[0] = CX + sg * (p[0] - CX);
        q[1] = CY + sg * (p[1] - CY);
    }
}

void orc_deform_inv(int kind, double s, const double q[3], double p[3]) {
    if (kind == ORC_TWIST_BEND) {
        double t[3];
        orc_deform_inv(ORC_BEND, s, q, t);
        orc_deform_inv(ORC_TWIST, s, t, p);
        return;
    }
    p[0] = q[0]; p[1] = q[1]; p[2] = q[2];
    if (kind == ORC_TWIST) {
        double th = 0.6 * s * q[2];       /* z is unchanged, so the angle is known */
        double x = q[0] - CX, y = q[1] - CY;
        p[0] = CX + cos(th) * x + sin(th) * y;
        p[1] = CY - sin(th) * x + cos(th) * y;
    } else if (kind == ORC_BEND) {
        double k = s / 1.5;
        if (k == 0.0) return;
        double ax = CX + 1.0 / k - q[0], az = q[2] - CZ;
        double rho = sqrt(ax * ax + az * az);
        double ph = atan2(az, ax);
        p[0] = CX + 1.0 / k - rho;
        p[2] = CZ + ph / k;
    } else if (kind == ORC_TAPER) {
        double sg = 1.0 - 0.5 * s * q[2];
        p[0] = CX + (q[0] - CX) / sg;
        p[1] = CY + (q[1] - CY) / sg;
    }
}

double orc_deform_jacdet(int kind, double s, const double p[3]) {
    if (kind == ORC_TWIST_BEND) {                 /* det of a product: twist (1) times bend at twist(p) */
        double t[3];
        orc_deform(ORC_TWIST, s, p, t);
        return orc_deform_jacdet(ORC_TWIST, s, p) * orc_deform_jacdet(ORC_BEND, s, t);
    }
    if (kind == ORC_BEND) return 1.0 - (s / 1.5) * (p[0] - CX);
    if (kind == ORC_TAPER) { double sg = 1.0 - 0.5 * s * p[2]; return sg * sg; }
    return 1.0;
}

/* Unit normal of the deformed surface at D(p), from the rest-space normal n at p. */
void orc_deform_normal(int kind, double s, const double p[3], const double n[3], double out[3]) {
    const double h = 1e-6;
    double J[3][3];
    for (int c = 0; c < 3; ++c) {
        double a[3] = {p[0], p[1], p[2]}, b[3] = {p[0], p[1], p[2]}, qa[3], qb[3];
        a[c] += h; b[c] -= h;
        orc_deform(kind, s, a, qa);
        orc_deform(kind, s, b, qb);
        for (int r = 0; r < 3; ++r) J[r][c] = (qa[r] - qb[r]) / (2.0 * h);
    }
    /* inverse by adjugate / determinant */
    double A[3][3];
    A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
    double v[3];
    for (int r = 0; r < 3; ++r) {           /* (J^-1)^T n: row r of the transpose = column r of J^-1 */
        v[r] = 0.0;
        for (int k = 0; k < 3; ++k) v[r] += (A[k][r] / det) * n[k];
    }
    double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int r = 0; r < 3; ++r) out[r] = l > 0.0 ? v[r] / l : 0.0;
}
