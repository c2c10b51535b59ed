/*
 * Oracle (test infrastructure only): hybrid encoding, intersection MLP, first-hit query,
 * multi-task loss with its analytic gradient, and Adam, in FP64.
 *
 * Passages followed:
 *  - Encoding, Eq. (1) and "Combining Positional Encoding with the Grid Encoding":
 *    gamma(x) = [x, sin(2^k x), cos(2^k x)] for k < F; the multi-level hash grid phi
 *    interpolates features from the neighbouring vertices of each level and concatenates
 *    the levels; the composite psi = phi(gamma(x)) runs phi on every PE sample separately.
 *    Readings: x is clamped to [0,1]^3 and the sin/cos samples are mapped to [0,1] by
 *    (v+1)/2 (the grid takes normalized points); one table set serves every sample; the
 *    hash is the Instant-NGP spatial hash (the grid encoding LSNIF builds on), dense
 *    indexing where (N_l+1)^3 fits the table.
 *  - Network and heads, Methodology and "Uncertainty-Weighted Multi-Task Loss": the
 *    encoded entry and exit points feed an MLP predicting occlusion, distance (ReLU),
 *    normal, albedo (sigmoid) and material.
 *  - Query, "Segmented Ray Distance Accumulation": segments are visited front to back and
 *    the first voxel with a predicted hit ends the ray; D = sum(delta_j + l_j) + delta_k + t_k,
 *    which for consecutive segments of one straight ray telescopes to t_in + local distance.
 *  - Loss, "Uncertainty-Weighted Multi-Task Loss": regression 0.5 exp(-s) L + 0.5 s,
 *    classification exp(-s) L + 0.5 s; log-space MSE for distance, cosine loss for normals,
 *    L1 on sigmoid albedo, cross-entropy for material and occlusion.
 *  - Concatenated encoding (the other reading of Eq. (1)): with concat_encoding the grid runs
 *    on the point itself and the raw gamma values are appended: [phi(x0), phi(x1), gamma(x0),
 *    gamma(x1)].
 *  - Per-sample tables (the other reading of one table set serving every sample of Eq. (1)):
 *    with per_sample_tables, PE sample s reads table set s, laid out [set][level][T][Fd].
 *  - Ablation switches, "Accuracy Comparison without Deformation" (Table 1) and the loss
 *    section's remark that the sigmoid distance output was replaced: dist_head = 1 restores
 *    a bounded head, sigma(z1) read as the hit's fraction of the rest segment and regressed
 *    by MSE against t* / l (clamped to [0,1]); fixed_weights = 1 drops the uncertainty
 *    weighting (every task weighs 1, s is not used and gets no gradient).  F = 0 removes the
 *    positional encoding.  Readings: the paper names the baselines' parts but not their
 *    formulas; these are the plainest forms consistent with that description.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define DIST_EPS 1e-4

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }
static double sigmoid(double v) { return 1.0 / (1.0 + exp(-v)); }

/* PE samples that go through the grid: all 1 + 2F of them for psi = phi(gamma(x)), only x
   itself for the concatenated [gamma, phi] reading. */
static int n_samples(const orc_model* m) { return m->concat_encoding ? 1 : 1 + 2 * m->pe_freqs; }
/* Raw gamma values per point that the concatenated reading appends: 3 (1 + 2F). */
static int gamma_width(const orc_model* m) { return m->concat_encoding ? 3 * (1 + 2 * m->pe_freqs) : 0; }
/* Table set of PE sample s: one set shared by all samples, or one per sample. */
static int table_set(const orc_model* m, int s) { return m->per_sample_tables ? s : 0; }
static int point_width(const orc_model* m) { return n_samples(m) * m->levels * m->feat_dim; }

/* Sample s of gamma(x) for one coordinate, and its derivative d sample / d x. */
static double pe_sample(int s, double x, double* dsdx) {
    if (s == 0) { *dsdx = 1.0; return x; }
    int k = (s - 1) / 2;
    double f = ldexp(1.0, k);
    if ((s - 1) % 2 == 0) { *dsdx = 0.5 * f * cos(f * x); return 0.5 * (sin(f * x) + 1.0); }
    *dsdx = -0.5 * f * sin(f * x);
    return 0.5 * (cos(f * x) + 1.0);
}

static uint32_t grid_index(const orc_model* m, int l, const uint32_t v[3]) {
    uint32_t n1 = (uint32_t)m->res[l] + 1u;
    uint32_t T = 1u << m->log2_table;
    if ((uint64_t)n1 * n1 * n1 <= T) return v[0] + n1 * (v[1] + n1 * v[2]);
    uint32_t h = (v[0] * 1u) ^ (v[1] * 2654435761u) ^ (v[2] * 805459861u);
    return h & (T - 1u);
}

/* Cell and weights of one sample at level l. */
static void grid_cell(const orc_model* m, int l, const double S[3], uint32_t i0[3], double w[3]) {
    int N = m->res[l];
    for (int a = 0; a < 3; ++a) {
        double pos = S[a] * N;
        double f = floor(pos);
        if (f > N - 1) f = N - 1;
        i0[a] = (uint32_t)f;
        w[a] = pos - f;
    }
}

void orc_encode_point(const orc_model* m, const double* tables, const double xin[3], double* out) {
    const int L = m->levels, Fd = m->feat_dim, S = n_samples(m);
    const int64_t T = 1LL << m->log2_table;
    double x[3] = {clamp01(xin[0]), clamp01(xin[1]), clamp01(xin[2])};
    for (int s = 0; s < S; ++s) {
        double smp[3], dd;
        for (int a = 0; a < 3; ++a) smp[a] = pe_sample(s, x[a], &dd);
        for (int l = 0; l < L; ++l) {
            uint32_t i0[3];
            double w[3];
            grid_cell(m, l, smp, i0, w);
            double* o = out + ((int64_t)s * L + l) * Fd;
            for (int f = 0; f < Fd; ++f) o[f] = 0.0;
            for (int c = 0; c < 8; ++c) {
                uint32_t v[3];
                double wt = 1.0;
                for (int a = 0; a < 3; ++a) {
                    int bit = (c >> a) & 1;
                    v[a] = i0[a] + bit;
                    wt *= bit ? w[a] : 1.0 - w[a];
                }
                const double* e = tables + (((int64_t)table_set(m, s) * L + l) * T + grid_index(m, l, v)) * Fd;
                for (int f = 0; f < Fd; ++f) o[f] += wt * e[f];
            }
        }
    }
}

/* Backward of one point's encoding: accumulates d tables and (optionally) d x. */
static void encode_point_backward(const orc_model* m, const double* tables, const double xin[3],
                                  const double* dout, double* gtab, double* gx) {
    const int L = m->levels, Fd = m->feat_dim, S = n_samples(m);
    const int64_t T = 1LL << m->log2_table;
    double x[3], inside[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = clamp01(xin[a]);
        inside[a] = (xin[a] >= 0.0 && xin[a] <= 1.0) ? 1.0 : 0.0;
    }
    double gacc[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < S; ++s) {
        double smp[3], dsdx[3];
        for (int a = 0; a < 3; ++a) smp[a] = pe_sample(s, x[a], &dsdx[a]);
        for (int l = 0; l < L; ++l) {
            uint32_t i0[3];
            double w[3];
            grid_cell(m, l, smp, i0, w);
            const double* g = dout + ((int64_t)s * L + l) * Fd;
            double dw[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 8; ++c) {
                uint32_t v[3];
                double f1[3];
                for (int a = 0; a < 3; ++a) {
                    int bit = (c >> a) & 1;
                    v[a] = i0[a] + bit;
                    f1[a] = bit ? w[a] : 1.0 - w[a];
                }
                double wt = f1[0] * f1[1] * f1[2];
                int64_t base = (((int64_t)table_set(m, s) * L + l) * T + grid_index(m, l, v)) * Fd;
                double gdot = 0.0;
                for (int f = 0; f < Fd; ++f) {
                    if (gtab) gtab[base + f] += wt * g[f];
                    gdot += g[f] * tables[base + f];
                }
                for (int a = 0; a < 3; ++a) {
                    double sgn = ((c >> a) & 1) ? 1.0 : -1.0;
                    dw[a] += gdot * sgn * f1[(a + 1) % 3] * f1[(a + 2) % 3];
                }
            }
            for (int a = 0; a < 3; ++a) gacc[a] += dw[a] * m->res[l] * dsdx[a];
        }
    }
    if (gx) for (int a = 0; a < 3; ++a) gx[a] += gacc[a] * inside[a];
}

/* Affine layers with ReLU between them (none after the last).  acts receives the input of
   every layer (acts[0] = the encoding) when non-null; z the output of the last layer. */
void orc_mlp_forward(const orc_model* m, const double* params, const double* in, double* z,
                     double* acts) {
    int maxw = 0;
    for (int j = 0; j <= m->n_layers; ++j) if (m->dims[j] > maxw) maxw = m->dims[j];
    double* cur = (double*)malloc(sizeof(double) * maxw);
    double* nxt = (double*)malloc(sizeof(double) * maxw);
    memcpy(cur, in, sizeof(double) * m->dims[0]);
    const double* p = params;
    int64_t aoff = 0;
    for (int j = 0; j < m->n_layers; ++j) {
        int ni = m->dims[j], no = m->dims[j + 1];
        if (acts) { memcpy(acts + aoff, cur, sizeof(double) * ni); aoff += ni; }
        const double* W = p;
        const double* b = p + (int64_t)no * ni;
        for (int r = 0; r < no; ++r) {
            double acc = b[r];
            for (int c = 0; c < ni; ++c) acc += W[(int64_t)r * ni + c] * cur[c];
            nxt[r] = (j + 1 < m->n_layers && acc < 0.0) ? 0.0 : acc;
        }
        p += (int64_t)no * ni + no;
        double* t = cur; cur = nxt; nxt = t;
    }
    memcpy(z, cur, sizeof(double) * m->dims[m->n_layers]);
    free(cur); free(nxt);
}

/* Conditioning of the hit logit: |b| + sum |w||h| of the last layer's row 0. */
static double hit_logit_scale(const orc_model* m, const double* params, const double* acts) {
    const double* p = params;
    int64_t aoff = 0;
    for (int j = 0; j + 1 < m->n_layers; ++j) {
        p += (int64_t)m->dims[j + 1] * m->dims[j] + m->dims[j + 1];
        aoff += m->dims[j];
    }
    int ni = m->dims[m->n_layers - 1], no = m->dims[m->n_layers];
    double s = fabs(p[(int64_t)no * ni]);
    for (int c = 0; c < ni; ++c) s += fabs(p[c] * acts[aoff + c]);
    return s;
}

static int64_t acts_width(const orc_model* m) {
    int64_t s = 0;
    for (int j = 0; j < m->n_layers; ++j) s += m->dims[j];
    return s;
}

/* gamma(x) of Eq. (1) as raw values on the clamped point: value 3 s + a is sample s of
   coordinate a (s = 0: x; s = 2k + 1: sin 2^k x; s = 2k + 2: cos 2^k x), and its derivative. */
static void gamma_raw(const orc_model* m, const double xin[3], double* out, double* dout) {
    for (int s = 0; s < 1 + 2 * m->pe_freqs; ++s)
        for (int a = 0; a < 3; ++a) {
            double x = clamp01(xin[a]), v, dv;
            if (s == 0) { v = x; dv = 1.0; }
            else {
                double f = ldexp(1.0, (s - 1) / 2);
                if ((s - 1) % 2 == 0) { v = sin(f * x); dv = f * cos(f * x); }
                else { v = cos(f * x); dv = -f * sin(f * x); }
            }
            out[3 * s + a] = v;
            if (dout) dout[3 * s + a] = dv;
        }
}

/* MLP input of a segment: psi(x0) ++ psi(x1), or with the concatenated reading
   phi(x0) ++ phi(x1) ++ gamma(x0) ++ gamma(x1). */
static void features(const orc_model* m, const double* tables, const double x0[3],
                     const double x1[3], double* enc) {
    orc_encode_point(m, tables, x0, enc);
    orc_encode_point(m, tables, x1, enc + point_width(m));
    if (m->concat_encoding) {
        gamma_raw(m, x0, enc + 2 * point_width(m), NULL);
        gamma_raw(m, x1, enc + 2 * point_width(m) + gamma_width(m), NULL);
    }
}

/* ------------------------------------------------------------------ batch entry points */

/* Threads of the OpenMP loops below (n <= 0: the runtime's default); returns the count in use. */
int32_t orc_set_threads(int32_t n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

void orc_deform_batch(int32_t kind, double s, int64_t n, const double* p, double* q, int32_t inverse) {
    for (int64_t i = 0; i < n; ++i) {
        if (inverse) orc_deform_inv(kind, s, p + 3 * i, q + 3 * i);
        else orc_deform(kind, s, p + 3 * i, q + 3 * i);
    }
}

void orc_jacdet_batch(int32_t kind, double s, int64_t n, const double* p, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = orc_deform_jacdet(kind, s, p + 3 * i);
}

void orc_scene_f_batch(int32_t kind, const double* sp, int64_t n, const double* p, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = orc_scene_f(kind, sp, p + 3 * i);
}

void orc_scene_grad_batch(int32_t kind, const double* sp, int64_t n, const double* p, double* g) {
    for (int64_t i = 0; i < n; ++i) orc_scene_grad(kind, sp, p + 3 * i, g + 3 * i);
}

void orc_scene_attr_batch(int32_t kind, const double* sp, int64_t n, const double* p, double* albedo,
                          int32_t* material) {
    for (int64_t i = 0; i < n; ++i) orc_scene_attr(kind, sp, p + 3 * i, albedo + 3 * i, material + i);
}

void orc_label_batch(int32_t kind, const double* sp, int32_t force_march, int64_t n,
                     const double* x0, const double* x1, uint8_t* hit, double* t, double* nrm,
                     double* alb, int32_t* mat) {
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i)
        orc_label(kind, sp, force_march, x0 + 3 * i, x1 + 3 * i, hit + i, t + i, nrm + 3 * i,
                  alb + 3 * i, mat + i);
}

/* Hit lists of n rays (o, d as n x 3): segments of ray i at [i*max_out, ...). */
void orc_trace_batch(int32_t N, const uint8_t* occ, const double* V, int64_t n, const double* o,
                     const double* d, int32_t brute, int32_t max_out, int32_t* cell, double* tin,
                     double* tout, int32_t* count, int32_t* flags, double* cin, double* cout) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        count[i] = orc_hitlist(N, occ, V, o + 3 * i, d + 3 * i, brute, max_out, cell + i * max_out,
                               tin + i * max_out, tout + i * max_out, flags ? flags + i : NULL,
                               cin ? cin + i * max_out : NULL, cout ? cout + i * max_out : NULL);
}

void orc_encode_batch(const orc_model* m, const double* tables, int64_t n, const double* x,
                      double* out) {
    const int W = point_width(m);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) orc_encode_point(m, tables, x + 3 * i, out + i * W);
}

/* Sparse Jacobian of the encoding with respect to the tables: for each of n points, every
   PE sample s, level l and corner c in the order of orc_encode_point, the flat index of the
   table entry the corner reads ((set L + l) T + entry; times feat_dim gives its first
   feature) and the corner's trilinear weight.  idx, w: [n][S][L][8]. */
void orc_encode_corners_batch(const orc_model* m, int64_t n, const double* xin, int64_t* idx, double* w) {
    const int L = m->levels, S = n_samples(m);
    const int64_t T = 1LL << m->log2_table;
    for (int64_t i = 0; i < n; ++i) {
        double x[3] = {clamp01(xin[3 * i]), clamp01(xin[3 * i + 1]), clamp01(xin[3 * i + 2])};
        for (int s = 0; s < S; ++s) {
            double smp[3], dd;
            for (int a = 0; a < 3; ++a) smp[a] = pe_sample(s, x[a], &dd);
            for (int l = 0; l < L; ++l) {
                uint32_t i0[3];
                double f[3];
                grid_cell(m, l, smp, i0, f);
                const int64_t o = ((i * S + s) * L + l) * 8;
                for (int c = 0; c < 8; ++c) {
                    uint32_t v[3];
                    double wt = 1.0;
                    for (int a = 0; a < 3; ++a) {
                        int bit = (c >> a) & 1;
                        v[a] = i0[a] + bit;
                        wt *= bit ? f[a] : 1.0 - f[a];
                    }
                    idx[o + c] = ((int64_t)table_set(m, s) * L + l) * T + grid_index(m, l, v);
                    w[o + c] = wt;
                }
            }
        }
    }
}

/* Adjoint of the encoding with respect to the tables (the table part of step 12's
   gradient): for each of n points, the rows dout[i] of d loss / d psi(x_i) are scattered
   into g_tables with the trilinear weights of every sample and level, exactly as the
   loss gradient does it.  The encoding is linear in the tables, so this is J^T dout. */
void orc_encode_backward_batch(const orc_model* m, const double* tables, int64_t n, const double* x,
                               const double* dout, double* g_tables) {
    const int W = point_width(m);
    for (int64_t i = 0; i < n; ++i) encode_point_backward(m, tables, x + 3 * i, dout + i * W, g_tables, NULL);
}

/* Network on given rest-space point pairs: z[i] = MLP(psi(x0_i) ++ psi(x1_i)). */
void orc_forward_batch(const orc_model* m, const double* tables, const double* params, int64_t n,
                       const double* x0, const double* x1, double* z, double* zscale) {
    const int E = m->dims[0], H = m->dims[m->n_layers];
    #pragma omp parallel
    {
        double* enc = (double*)malloc(sizeof(double) * E);
        double* acts = (double*)malloc(sizeof(double) * acts_width(m));
        #pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            features(m, tables, x0 + 3 * i, x1 + 3 * i, enc);
            orc_mlp_forward(m, params, enc, z + i * H, acts);
            if (zscale) zscale[i] = hit_logit_scale(m, params, acts);
        }
        free(enc); free(acts);
    }
}

/* First-hit query of n rays under one pose.  Per ray: hit, distance D along the ray,
   rest-space hit point, normal, albedo, material, voxel, hit logit, segments evaluated,
   and the smallest relative margin |z0| / scale among the evaluated segments.
   dnrm (nullable): the normal carried to deformed space, (J^-1)^T n at the rest hit point.
   tmax (nullable, per ray): the occlusion form of the query used for shadow rays, the
   renderer integration the introduction and conclusion describe: voxels entered at
   t_in >= tmax are not visited, and a first hit at D >= tmax is a miss. */
void orc_query_batch(const orc_model* m, const double* tables, const double* params, int32_t N,
                     const uint8_t* occ, int32_t kind, double s, int64_t n, const double* o,
                     const double* d, uint8_t* hit, double* tout_ray, double* xrest, double* nrm,
                     double* alb, int32_t* mat, int32_t* cell_out, double* logit, int32_t* nq,
                     double* margin, double* zhit, double* seginfo, const double* tmax,
                     double* dnrm) {
    const int E = m->dims[0], H = m->dims[m->n_layers], M = m->n_materials;
    double* V = (double*)malloc(sizeof(double) * 3 * (size_t)(N + 1) * (N + 1) * (N + 1));
    orc_lattice_vertices(kind, s, N, V);
    const int cap = 16 * N + 64;
    #pragma omp parallel
    {
        int32_t* cells = (int32_t*)malloc(sizeof(int32_t) * cap);
        double* tin = (double*)malloc(sizeof(double) * cap);
        double* tou = (double*)malloc(sizeof(double) * cap);
        double* cin = (double*)malloc(sizeof(double) * cap);
        double* cou = (double*)malloc(sizeof(double) * cap);
        double* enc = (double*)malloc(sizeof(double) * E);
        double* acts = (double*)malloc(sizeof(double) * acts_width(m));
        double* z = (double*)malloc(sizeof(double) * H);
        #pragma omp for schedule(dynamic, 8)
        for (int64_t r = 0; r < n; ++r) {
            const double* ro = o + 3 * r;
            const double* rd = d + 3 * r;
            int32_t ns = orc_hitlist(N, occ, V, ro, rd, 0, cap, cells, tin, tou, NULL, cin, cou);
            if (ns > cap) ns = cap;
            hit[r] = 0; tout_ray[r] = INFINITY; cell_out[r] = -1; mat[r] = -1;
            logit[r] = -INFINITY; nq[r] = 0; margin[r] = INFINITY;
            for (int a = 0; a < 3; ++a) { xrest[3 * r + a] = 0; nrm[3 * r + a] = 0; alb[3 * r + a] = 0; }
            const double tm = tmax ? tmax[r] : INFINITY;
            for (int k = 0; k < ns; ++k) {
                if (tin[k] >= tm) break;
                double p0[3], p1[3], x0[3], x1[3];
                for (int a = 0; a < 3; ++a) { p0[a] = ro[a] + tin[k] * rd[a]; p1[a] = ro[a] + tou[k] * rd[a]; }
                orc_deform_inv(kind, s, p0, x0);
                orc_deform_inv(kind, s, p1, x1);
                features(m, tables, x0, x1, enc);
                orc_mlp_forward(m, params, enc, z, acts);
                nq[r] = k + 1;
                logit[r] = z[0];
                double sc = hit_logit_scale(m, params, acts);
                double mg = sc > 0.0 ? fabs(z[0]) / sc : INFINITY;
                if (mg < margin[r]) margin[r] = mg;
                if (!(z[0] > 0.0)) continue;
                double e[3] = {x1[0] - x0[0], x1[1] - x0[1], x1[2] - x0[2]};
                double lr = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
                double f;
                if (m->dist_head == 1) {
                    f = sigmoid(z[1]);
                } else {
                    double dh = z[1] > 0.0 ? z[1] : 0.0;
                    f = lr > 0.0 ? clamp01(dh / lr) : 0.0;
                }
                double D = tin[k] + f * (tou[k] - tin[k]);
                if (D >= tm) break;                 /* the first hit lies beyond tmax */
                hit[r] = 1;
                tout_ray[r] = D;
                for (int a = 0; a < 3; ++a) xrest[3 * r + a] = x0[a] + f * e[a];
                double nl = sqrt(z[2] * z[2] + z[3] * z[3] + z[4] * z[4]);
                if (nl < 1e-12) nl = 1e-12;
                for (int a = 0; a < 3; ++a) { nrm[3 * r + a] = z[2 + a] / nl; alb[3 * r + a] = sigmoid(z[5 + a]); }
                if (dnrm) orc_deform_normal(kind, s, xrest + 3 * r, nrm + 3 * r, dnrm + 3 * r);
                if (M == 1) mat[r] = z[8] > 0.0 ? 1 : 0;
                else {
                    int best = 0;
                    for (int c = 1; c < M; ++c) if (z[8 + c] > z[8 + best]) best = c;
                    mat[r] = best;
                }
                cell_out[r] = cells[k];
                if (zhit) for (int h = 0; h < H; ++h) zhit[r * H + h] = z[h];
                if (seginfo) {
                    double* si = seginfo + 5 * r;
                    si[0] = tin[k]; si[1] = tou[k]; si[2] = lr; si[3] = cin[k]; si[4] = cou[k];
                }
                break;
            }
        }
        free(cells); free(tin); free(tou); free(cin); free(cou); free(enc); free(acts); free(z);
    }
    free(V);
}

/* Multi-task loss over a batch and its gradient with respect to every parameter.
   Task order: hit, distance, normal, albedo, material; s holds log sigma^2 per task.
   losses[0..4] = per-task batch losses, losses[5] = weighted total.  Gradients are added
   to the g_* arrays (which the caller zeroes); g_x0 / g_x1 may be null. */
void orc_loss_grad(const orc_model* m, const double* tables, const double* params, const double* s,
                   int64_t B, const double* x0, const double* x1, const uint8_t* lhit,
                   const double* lt, const double* ln, const double* la, const int32_t* lm,
                   double* losses, double* g_tables, double* g_params, double* g_s, double* g_x0,
                   double* g_x1, double* dz_out, int32_t fixed_weights) {
    const int E = m->dims[0], H = m->dims[m->n_layers], M = m->n_materials, PW = point_width(m);
    int64_t P = 0;
    for (int64_t i = 0; i < B; ++i) P += lhit[i] ? 1 : 0;
    double w[5];
    w[0] = exp(-s[0]);              /* classification */
    w[1] = 0.5 * exp(-s[1]);        /* regression */
    w[2] = 0.5 * exp(-s[2]);
    w[3] = 0.5 * exp(-s[3]);
    w[4] = exp(-s[4]);              /* classification */
    if (fixed_weights)
        for (int k = 0; k < 5; ++k) w[k] = 1.0;
    double sum[5] = {0, 0, 0, 0, 0};
    double* enc = (double*)malloc(sizeof(double) * E);
    double* acts = (double*)malloc(sizeof(double) * acts_width(m));
    double* z = (double*)malloc(sizeof(double) * H);
    double* dz = (double*)malloc(sizeof(double) * H);
    int maxw = 0;
    for (int j = 0; j <= m->n_layers; ++j) if (m->dims[j] > maxw) maxw = m->dims[j];
    double* dcur = (double*)malloc(sizeof(double) * maxw);
    double* dprev = (double*)malloc(sizeof(double) * maxw);
    for (int64_t i = 0; i < B; ++i) {
        features(m, tables, x0 + 3 * i, x1 + 3 * i, enc);
        orc_mlp_forward(m, params, enc, z, acts);
        for (int h = 0; h < H; ++h) dz[h] = 0.0;
        /* occlusion: binary cross-entropy with logits over the whole batch */
        double y = lhit[i] ? 1.0 : 0.0;
        sum[0] += (z[0] > 0 ? z[0] : 0.0) - z[0] * y + log1p(exp(-fabs(z[0])));
        dz[0] = w[0] * (sigmoid(z[0]) - y) / (double)B;
        if (lhit[i] && P > 0) {
            if (m->dist_head == 1) {
                /* distance: MSE of the sigmoid fraction against t* / l of the rest segment */
                const double* a0 = x0 + 3 * i;
                const double* a1 = x1 + 3 * i;
                double e[3] = {a1[0] - a0[0], a1[1] - a0[1], a1[2] - a0[2]};
                double lr = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
                double tau = lr > 0.0 ? clamp01(lt[i] / lr) : 0.0;
                double p = sigmoid(z[1]);
                double r = p - tau;
                sum[1] += r * r;
                dz[1] = w[1] * 2.0 * r * p * (1.0 - p) / (double)P;
            } else {
                /* distance: MSE of logs, ReLU output */
                double dh = z[1] > 0.0 ? z[1] : 0.0;
                double r = log(dh + DIST_EPS) - log(lt[i] + DIST_EPS);
                sum[1] += r * r;
                if (z[1] > 0.0) dz[1] = w[1] * 2.0 * r / (dh + DIST_EPS) / (double)P;
            }
            /* normal: 1 - cosine */
            const double* nt = ln + 3 * i;
            double v[3] = {z[2], z[3], z[4]};
            double vl = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            double den = vl > 1e-12 ? vl : 1e-12;
            double nh[3] = {v[0] / den, v[1] / den, v[2] / den};
            double c = nh[0] * nt[0] + nh[1] * nt[1] + nh[2] * nt[2];
            sum[2] += 1.0 - c;
            for (int a = 0; a < 3; ++a) {
                double g = vl > 1e-12 ? -(nt[a] - nh[a] * c) / vl : -nt[a] / 1e-12;
                dz[2 + a] = w[2] * g / (double)P;
            }
            /* albedo: L1 on sigmoid outputs, mean over the three channels */
            for (int a = 0; a < 3; ++a) {
                double ah = sigmoid(z[5 + a]);
                double df = ah - la[3 * i + a];
                sum[3] += fabs(df) / 3.0;
                double sg = df > 0 ? 1.0 : (df < 0 ? -1.0 : 0.0);
                dz[5 + a] = w[3] * sg * ah * (1.0 - ah) / (3.0 * (double)P);
            }
            /* material: softmax cross-entropy (binary for a single logit) */
            if (M == 1) {
                double ym = lm[i] ? 1.0 : 0.0;
                sum[4] += (z[8] > 0 ? z[8] : 0.0) - z[8] * ym + log1p(exp(-fabs(z[8])));
                dz[8] = w[4] * (sigmoid(z[8]) - ym) / (double)P;
            } else {
                double mx = z[8];
                for (int c2 = 1; c2 < M; ++c2) if (z[8 + c2] > mx) mx = z[8 + c2];
                double se = 0.0;
                for (int c2 = 0; c2 < M; ++c2) se += exp(z[8 + c2] - mx);
                double lse = mx + log(se);
                sum[4] += lse - z[8 + lm[i]];
                for (int c2 = 0; c2 < M; ++c2) {
                    double pr = exp(z[8 + c2] - lse);
                    dz[8 + c2] = w[4] * (pr - (c2 == lm[i] ? 1.0 : 0.0)) / (double)P;
                }
            }
        }
        if (dz_out) memcpy(dz_out + i * H, dz, sizeof(double) * H);
        /* backward through the MLP */
        memcpy(dcur, dz, sizeof(double) * H);
        int64_t poff = 0, aoff = 0;
        int64_t* po = (int64_t*)malloc(sizeof(int64_t) * m->n_layers);
        int64_t* ao = (int64_t*)malloc(sizeof(int64_t) * m->n_layers);
        for (int j = 0; j < m->n_layers; ++j) {
            po[j] = poff; ao[j] = aoff;
            poff += (int64_t)m->dims[j + 1] * m->dims[j] + m->dims[j + 1];
            aoff += m->dims[j];
        }
        for (int j = m->n_layers - 1; j >= 0; --j) {
            int ni = m->dims[j], no = m->dims[j + 1];
            const double* W = params + po[j];
            double* gW = g_params + po[j];
            double* gb = gW + (int64_t)no * ni;
            const double* hin = acts + ao[j];
            for (int r = 0; r < no; ++r) {
                gb[r] += dcur[r];
                for (int c = 0; c < ni; ++c) gW[(int64_t)r * ni + c] += dcur[r] * hin[c];
            }
            for (int c = 0; c < ni; ++c) {
                double acc = 0.0;
                for (int r = 0; r < no; ++r) acc += W[(int64_t)r * ni + c] * dcur[r];
                /* the input of hidden layers went through ReLU: zero where it was clipped */
                dprev[c] = (j > 0 && !(hin[c] > 0.0)) ? 0.0 : acc;
            }
            double* t = dcur; dcur = dprev; dprev = t;
        }
        free(po); free(ao);
        /* dcur now holds d loss / d encoding */
        encode_point_backward(m, tables, x0 + 3 * i, dcur, g_tables, g_x0 ? g_x0 + 3 * i : NULL);
        encode_point_backward(m, tables, x1 + 3 * i, dcur + PW, g_tables, g_x1 ? g_x1 + 3 * i : NULL);
        if (m->concat_encoding) {        /* gamma part: d x_a += d gamma * d gamma / d x_a inside the cube */
            const int GW = gamma_width(m);
            double* val = (double*)malloc(sizeof(double) * GW);
            double* der = (double*)malloc(sizeof(double) * GW);
            for (int p = 0; p < 2; ++p) {
                const double* xp = (p ? x1 : x0) + 3 * i;
                double* gx = p ? (g_x1 ? g_x1 + 3 * i : NULL) : (g_x0 ? g_x0 + 3 * i : NULL);
                if (!gx) continue;
                gamma_raw(m, xp, val, der);
                const double* dg = dcur + 2 * PW + p * GW;
                for (int v = 0; v < GW; ++v) {
                    const int a = v % 3;
                    if (xp[a] >= 0.0 && xp[a] <= 1.0) gx[a] += dg[v] * der[v];
                }
            }
            free(val); free(der);
        }
    }
    double Ls[5];
    Ls[0] = sum[0] / (double)B;
    for (int k = 1; k < 5; ++k) Ls[k] = P > 0 ? sum[k] / (double)P : 0.0;
    double total = 0.0;
    for (int k = 0; k < 5; ++k) {
        if (fixed_weights) {
            total += Ls[k];
        } else {
            total += w[k] * Ls[k] + 0.5 * s[k];
            g_s[k] += -w[k] * Ls[k] + 0.5;
        }
        losses[k] = Ls[k];
    }
    losses[5] = total;
    free(enc); free(acts); free(z); free(dz); free(dcur); free(dprev);
}

/* One Adam step with bias correction (the torch.optim.Adam update, no weight decay). */
void orc_adam(int64_t n, double* theta, const double* g, double* mo, double* ve, int32_t step,
              double lr, double b1, double b2, double eps) {
    double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    for (int64_t i = 0; i < n; ++i) {
        mo[i] = b1 * mo[i] + (1.0 - b1) * g[i];
        ve[i] = b2 * ve[i] + (1.0 - b2) * g[i] * g[i];
        double mh = mo[i] / c1, vh = ve[i] / c2;
        theta[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
