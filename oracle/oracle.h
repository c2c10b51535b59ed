/*
 * FP64 CPU oracle of the deformation-aware neural intersection function.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or call
 * this code; only the tests, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no code, header or constant table with the GPU library.
 *
 * Every routine is a plain, slow, step-by-step restatement of the method as the paper
 * describes it (section names cited at each definition), in double precision.
 */
#ifndef NIF_ORACLE_H
#define NIF_ORACLE_H
#include <stdint.h>

#define ORC_IDENTITY 0
#define ORC_TWIST 1
#define ORC_BEND 2
#define ORC_TAPER 3
#define ORC_TWIST_BEND 4

#define ORC_SCENE_TORUS 0
#define ORC_SCENE_SPHERES 1
#define ORC_SCENE_BLOBS 2

/* Hyper-parameters of the encoding and the MLP (plain values, no derived state). */
typedef struct {
    int32_t levels, log2_table, feat_dim, pe_freqs;
    int32_t res[32];
    int32_t n_layers;      /* number of affine layers (hidden layers + output layer) */
    int32_t dims[16];      /* dims[0] = encoding width, dims[n_layers] = head count  */
    int32_t n_materials;
    int32_t dist_head;     /* 0: ReLU rest-space distance, log-space MSE (the paper's head);
                              1: sigmoid fraction of the rest segment, MSE (the bounded head
                              the paper replaces, kept as an ablation switch) */
    int32_t per_sample_tables; /* 0: one table set for every PE sample; 1: set s for sample s */
    int32_t concat_encoding;   /* 0: psi = phi(gamma(x)); 1: [phi(x), gamma(x)] (raw gamma) */
} orc_model;

/* deform.c */
void orc_deform(int kind, double s, const double p[3], double q[3]);
void orc_deform_inv(int kind, double s, const double q[3], double p[3]);
double orc_deform_jacdet(int kind, double s, const double p[3]);
void orc_deform_normal(int kind, double s, const double p[3], const double n[3], double out[3]);

/* scene.c */
double orc_scene_f(int kind, const double* sp, const double p[3]);
void orc_scene_grad(int kind, const double* sp, const double p[3], double g[3]);
void orc_scene_attr(int kind, const double* sp, const double p[3], double albedo[3], int32_t* material);
void orc_voxelize(int kind, const double* sp, int32_t N, uint8_t* occ);
void orc_label(int kind, const double* sp, int force_march, const double x0[3], const double x1[3],
               uint8_t* hit, double* t, double n[3], double a[3], int32_t* m);

/* lattice.c */
void orc_lattice_vertices(int kind, double s, int32_t N, double* V);
int32_t orc_hitlist(int32_t N, const uint8_t* occ, const double* V, const double o[3], const double d[3],
                    int32_t brute, int32_t max_out, int32_t* cell, double* tin, double* tout,
                    int32_t* flags, double* cin, double* cout);

/* network.c */
void orc_encode_point(const orc_model* m, const double* tables, const double x[3], double* out);
void orc_mlp_forward(const orc_model* m, const double* params, const double* in, double* z,
                     double* acts);
#endif
