/*
 * libnif -- deformation-aware neural intersection function on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the data-parallel hot path of the method: per-ray neural intersection queries
 * under a parameterized deformation, and the training step of the network.
 *
 * Conventions shared by every entry point
 *  - Every function returns an int status: NIF_OK (0) or an error code > 0.  On error the
 *    call has enqueued nothing, and nif_last_error() returns a message for the calling
 *    thread.  No C++ exception crosses this boundary.
 *  - Pointers named *_dev are device pointers owned by the caller; pointers named *_host
 *    are host pointers read during the call only.  Buffers are contiguous and FP32 unless
 *    stated.  Rays and points are structure-of-arrays.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is enqueued on it
 *    and the call returns without synchronising, except where stated.  nif_backward and
 *    nif_train_step also run the table-gradient part of the backward on a stream the model
 *    owns, forked from `stream` and joined back to it with events before the call returns.
 *    Both may be captured into a HIP graph (the fork and join become graph edges); they
 *    clear their accumulators with kernels, not memset nodes.
 *  - Opaque handles (nif_model, nif_grid) own their device memory, which is allocated at
 *    create/build time only.  nif_query, nif_trace, nif_forward, nif_encode, nif_backward
 *    and nif_train_step never allocate device memory.  A handle must not be used by two
 *    streams at once.
 *  - Device-side conditions (segment-list overflow, non-finite loss) are reported through
 *    device buffers the caller reads after its own synchronisation.
 */
#ifndef NIF_H
#define NIF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    NIF_OK = 0,
    NIF_E_INVALID_ARG = 1,   /* null pointer, bad size, bad enum value */
    NIF_E_UNSUPPORTED = 2,   /* valid but not implemented (e.g. a layer width that is not a multiple of 16) */
    NIF_E_OOM = 3,           /* device allocation failed (create/build only) */
    NIF_E_DEVICE = 4,        /* a HIP runtime call failed */
    NIF_E_STATE = 5          /* handle not ready (e.g. parameters never set) */
};
const char* nif_status_string(int status);
const char* nif_last_error(void);
int nif_version(void);

typedef struct nif_model nif_model;
typedef struct nif_grid nif_grid;
typedef void* nif_stream;

/* ---------------------------------------------------------------- deformation
 * A pose is one parameterized deformation D of the rest space (Methodology: the network
 * lives in rest space; rays are traced in deformed space and mapped back through the
 * inverse deformation).  Kinds and strength s in [0, 1]; pivot at the cube centre c:
 *   TWIST: rotation about the z axis through c by 0.6 s z radians;
 *   BEND : circular bend in the x-z plane with curvature s / 1.5;
 *   TAPER: x, y scaled about c by 1 - 0.5 s z;
 *   TWIST_BEND: the twist followed by the bend, both at strength s (a composed pose).
 */
enum { NIF_DEFORM_IDENTITY = 0, NIF_DEFORM_TWIST = 1, NIF_DEFORM_BEND = 2, NIF_DEFORM_TAPER = 3,
       NIF_DEFORM_TWIST_BEND = 4 };
typedef struct { int32_t kind; float strength; } nif_pose;

/* ---------------------------------------------------------------- model
 * Hybrid encoding psi = phi(gamma(x)) of Eq. (1) (PE samples, each run through the
 * multiresolution hash grid) on the rest-space entry and exit points of a voxel segment,
 * followed by an MLP with ReLU hidden layers and 8 + n_materials outputs:
 * [hit logit, distance, normal(3), albedo(3), material logits].
 * Canonical FP32 parameter layouts (the ones nif_model_set_params takes):
 *   tables: [sets][levels][2^log2_table][feat_dim], sets = 1 + 2 pe_freqs with per_sample_tables
 *           else 1
 *   mlp   : per layer W[out][in] row-major then b[out]; layer widths
 *           E = 2 (1 + 2 pe_freqs) levels feat_dim (see concat_encoding for the other form),
 *           hidden_width x hidden_layers, 8 + n_materials
 *   s     : [5] log-variances of the tasks (hit, distance, normal, albedo, material)
 */
enum { NIF_TABLE_F32 = 0, NIF_TABLE_F16 = 1 };
enum { NIF_PREC_FP32 = 0, NIF_PREC_BF16 = 1, NIF_PREC_FP16 = 2 };
/* Distance head ("Uncertainty-Weighted Multi-Task Loss": the bounded sigmoid output is
 * replaced by a ReLU distance regressed in log space).
 *   NIF_DIST_LOG_RELU: d = ReLU(z1) is the rest-space distance from the segment's entry point;
 *                      the hit's fraction of the segment is clamp(d / l, 0, 1), l the rest length;
 *                      loss (log(d + 1e-4) - log(t* + 1e-4))^2.
 *   NIF_DIST_SIGMOID:  the ablation baseline: the fraction is sigmoid(z1) itself; loss
 *                      (sigmoid(z1) - clamp(t* / l, 0, 1))^2. */
enum { NIF_DIST_LOG_RELU = 0, NIF_DIST_SIGMOID = 1 };

typedef struct {
    int32_t levels;          /* L: 4, 8, 12 or 16 with feat_dim 2; even, 2..16 with feat_dim 3 */
    int32_t log2_table;      /* T = 2^log2_table entries per level, 4..24 */
    int32_t feat_dim;        /* features per level: 2, or 3 (the paper's comparison of deformation
                                results: two levels, base resolution 64, three features) */
    int32_t table_dtype;     /* NIF_TABLE_F32 or NIF_TABLE_F16 (working copy; master is FP32) */
    int32_t res[32];         /* per-level grid resolution N_l >= 1 */
    int32_t pe_freqs;        /* F >= 0: PE samples per point = 1 + 2F */
    int32_t hidden_width;    /* multiple of 16, <= 128 */
    int32_t hidden_layers;   /* 1..8 */
    int32_t n_materials;     /* 1..8 */
    int32_t dist_head;       /* NIF_DIST_LOG_RELU (the method) or NIF_DIST_SIGMOID (ablation) */
    int32_t per_sample_tables; /* 0: one table set serves every PE sample (Eq. (1) as read here);
                                  1: PE sample s reads its own set s; tables [sets][L][T][feat_dim] */
    int32_t concat_encoding; /* 0: psi = phi(gamma(x)) (Eq. (1) as read here); 1: the other reading,
                                the grid on x itself and the raw gamma values appended:
                                [phi(x0), phi(x1), gamma(x0), gamma(x1)], gamma value 3 s + a =
                                sample s (x, sin 2^k x, cos 2^k x) of axis a of the clamped point;
                                E = 2 (levels feat_dim + 3 (1 + 2 pe_freqs)); feat_dim 2 only */
} nif_model_desc;

/* Allocates parameters (FP32 masters and working copies), gradients and Adam state. */
int nif_model_create(const nif_model_desc* desc, nif_model** out);
int nif_model_destroy(nif_model* model);
/* Element counts of the canonical tables and MLP parameter vectors. */
int nif_model_sizes(const nif_model_desc* desc, int64_t* n_table, int64_t* n_mlp);
/* Copies canonical FP32 parameters in (device pointers; s_dev may be NULL = zeros) and
   refreshes the working copies (FP16 tables, padded FP32/BF16/FP16 MLP) by
   round-to-nearest-even.  Resets gradients, Adam moments and the step counter. */
int nif_model_set_params(nif_model* model, const float* tables_dev, const float* mlp_dev,
                         const float* s_dev, nif_stream stream);
/* Copies the FP32 masters out (any pointer may be NULL). */
int nif_model_get_params(const nif_model* model, float* tables_dev, float* mlp_dev, float* s_dev,
                         nif_stream stream);
/* Gradient accumulators (FP32, canonical layouts) filled by nif_backward / nif_train_step. */
int nif_model_get_grads(const nif_model* model, float* g_tables_dev, float* g_mlp_dev, float* g_s_dev,
                        nif_stream stream);
int nif_model_zero_grads(nif_model* model, nif_stream stream);
/* Allocates the training scratch for batches of up to max_batch samples (activations,
   deltas, a [min(max_batch, 2^17)][E] encoding scratch for the backward's recomputation,
   the table-gradient additions of a round of min(max_batch, 2^18) samples, weight-gradient
   partials and the spatially ordered copy of a batch); nif_backward and nif_train_step fail with NIF_E_STATE above it.  A later call
   with a larger max_batch frees and re-allocates everything, the stored encoding included. */
int nif_model_reserve(nif_model* model, int64_t max_batch);
/* Allocates the [max_batch][E] FP32 stored encoding that nif_train_step uses when
   nif_train_cfg.store_encoding = 1 (NIF_E_STATE before nif_model_reserve; idempotent). */
int nif_model_reserve_encoding(nif_model* model);

/* ---------------------------------------------------------------- scene preparation
 * Rest-space voxelization (Methodology: the geometry is voxelized in rest space).  Cell
 * (i,j,k) of the N^3 grid over [0,1]^3 is occupied iff the scene's implicit function,
 * sampled on the 5^3 sub-lattice of the closed cell, takes both signs.
 *   scene_kind 0 torus   params [cx,cy,cz,R,r]
 *              1 spheres params [n, (cx,cy,cz,r, ar,ag,ab, material) x n]
 *              2 blobs   params [n, (mx,my,mz,sigma, cr,cg,cb, material) x n]
 * occ_dev: u8[N^3], index i + N (j + N k).  Evaluated in FP32. */
int nif_voxelize(int32_t scene_kind, const double* params_host, int32_t n_params, int32_t N,
                 uint8_t* occ_dev, nif_stream stream);

/* Ground-truth labels of n rest-space segments [x0, x1] (x0_dev, x1_dev: SoA [3][n] FP32,
 * device) against the same analytic scene (Methodology: each locally linearized segment is
 * supervised with the rest geometry along its chord).  The label point is the first point of
 * the chord where f <= 0: the start if f(x0) <= 0; for spheres the smallest entering root of
 * the per-sphere quadratic in [0, |x1 - x0|] (unless force_march != 0); otherwise 256 uniform
 * sign steps and bisection of the first bracket down to 1e-13.  Outputs (device, each
 * nullable): hit u8[n]; t f32[n] distance from x0 (0 when no hit); normal f32 SoA [3][n]
 * = grad f / |grad f| at the point; albedo f32 SoA [3][n]; material i32[n] (torus: [x >= 1/2];
 * spheres: of the sphere with the smallest signed distance; blobs: of the largest
 * contribution, albedo = contribution-weighted colour); misses get zeros.  Evaluated in FP64.
 * Copies the parameters to the device and synchronises the stream. */
int nif_label(int32_t scene_kind, const double* params_host, int32_t n_params, int32_t force_march,
              const float* x0_dev, const float* x1_dev, int64_t n, uint8_t* hit_dev, float* t_dev,
              float* normal_dev, float* albedo_dev, int32_t* material_dev, nif_stream stream);
/* nif_label for callers that cannot allocate device memory (tight data-generation loops,
 * harnesses that forbid hipMalloc).  Same arguments and outputs as nif_label, bit for bit;
 * it allocates nothing and does not synchronise: the scene parameters are staged (copied
 * from params_host before the call returns) into a fixed per-device array of the library,
 * NIF_LABEL_NOALLOC_MAX_PARAMS doubles (32,832 bytes, held by every device the library runs
 * on until the process ends); more parameters are rejected with NIF_E_INVALID_ARG.  Every
 * call on one device shares that array: calls that overlap on a device (other streams or
 * threads, before the previous call's kernel has finished) race on it; calls on one stream
 * are ordered. */
#define NIF_LABEL_NOALLOC_MAX_PARAMS 4104
int nif_label_noalloc(int32_t scene_kind, const double* params_host, int32_t n_params, int32_t force_march,
                      const float* x0_dev, const float* x1_dev, int64_t n, uint8_t* hit_dev, float* t_dev,
                      float* normal_dev, float* albedo_dev, int32_t* material_dev, nif_stream stream);

/* ---------------------------------------------------------------- deformed grid
 * Per pose: the deformed lattice vertices V_ijk = D(i/N, j/N, k/N) (faces split along their
 * main diagonal), and an acceleration structure over the occupied deformed voxels
 * (Methodology, "Voxel Traversal under Deformation": voxel sizes vary under deformation, so
 * voxels are found by geometric tests rather than index arithmetic).  Here the structure is
 * a uniform bin grid over each pose's deformed bounding box; bins_per_axis = 0 picks N/2.
 * Synchronises `stream` (it sizes the bin lists on the host) and allocates.
 * occ_dev: u8[N^3] as above; poses_host: [n_poses]. */
int nif_build_grid(const uint8_t* occ_dev, int32_t N, const nif_pose* poses_host, int32_t n_poses,
                   int32_t bins_per_axis, nif_grid** out, nif_stream stream);
int nif_grid_destroy(nif_grid* grid);
/* Re-poses an existing grid (same occupancy, same pose count): new kinds/strengths, the
 * lattice vertices, bounding boxes, bin sizes and bin lists are recomputed on the device.
 * No allocation and no synchronisation.  The bin lists keep the capacity of the build plus
 * 50%; a pose whose lists would not fit is emptied (its rays miss) and the overflow flag of
 * nif_grid_info is set. */
int nif_grid_update(nif_grid* grid, const nif_pose* poses_host, int32_t n_poses, nif_stream stream);
/* Number of occupied voxels; bin-list entries of one pose at build time; overflow flag of the
 * last build/update (reading it synchronises the null stream).  Any pointer may be NULL. */
int nif_grid_info(const nif_grid* grid, int32_t pose, int64_t* n_occupied, int64_t* n_refs,
                  int32_t* overflow);
/* Deformed-space box of pose `pose`'s bin grid as of the last build/update: it holds every
 * occupied deformed voxel (FP32 lattice, padded by 1e-5 on each side).  lo[3], hi[3] are host arrays; a
 * pose with no occupied voxel gives lo = hi = 0.  Synchronises the null stream. */
int nif_grid_bounds(const nif_grid* grid, int32_t pose, float* lo, float* hi);

/* ---------------------------------------------------------------- rays
 * Deformed-space rays o + t d, grouped by pose: rays [pose_offsets[p], pose_offsets[p+1])
 * use pose p.  pose_offsets_dev: int64[n_poses + 1] on the device, pose_offsets[0] = 0 and
 * pose_offsets[n_poses] = n_rays.  d need not be unit; t is in units of |d|.
 * tmax: nullable float[n_rays] on the device (NULL = unbounded); used by nif_query only. */
typedef struct {
    const float *ox, *oy, *oz, *dx, *dy, *dz;
    const int64_t* pose_offsets;
    const float* tmax;
} nif_rays;

/* Ordered occupied-voxel segments of each ray (Methodology, "Segmented Ray Distance
 * Accumulation": entry/exit points of every occupied voxel the straight deformed ray
 * crosses).  Segment k of ray i is stored at i*max_seg + k: voxel id, t_in (clipped to
 * t >= 0), t_out, and the rest-space entry/exit points x0 = D^-1(o + t_in d),
 * x1 = D^-1(o + t_out d) as SoA [3][n_rays*max_seg].  count[i] is the full number of
 * segments (may exceed max_seg: only the first max_seg are stored).  Nullable: x0, x1. */
typedef struct {
    int32_t* count; int32_t* cell; float* t_in; float* t_out; float* x0; float* x1;
} nif_segments;
int nif_trace(const nif_grid* grid, const nif_rays* rays, int64_t n_rays, int32_t max_seg,
              const nif_segments* out, nif_stream stream);

/* ---------------------------------------------------------------- query
 * First-hit neural intersection query (the hot path).  Per ray: walk its occupied voxels
 * front to back; for each, map entry/exit to rest space, encode with psi, run the MLP;
 * the first voxel whose hit logit is > 0 ends the ray.  Its distance is
 * D = t_in + f (t_out - t_in), f = clamp(relu(z_dist) / |x1 - x0|, 0, 1) (the segmented
 * accumulation of the paper, which telescopes for one straight ray), its rest-space hit
 * point x0 + f (x1 - x0), normal z_n / |z_n|, albedo sigmoid(z_a), material argmax.
 * Misses: hit 0, t +inf, cell -1, material -1, other fields 0.
 * With rays->tmax (the occlusion query of shadow rays, for the renderer integration of the
 * introduction and conclusion): voxels entered at t_in >= tmax are not visited and a first
 * hit at D >= tmax is reported as a miss; pass only out->hit for a pure visibility bit.
 * Every output pointer is nullable (not written).  Outputs are indexed by ray. */
typedef struct {
    uint8_t* hit; float* t; float *nx, *ny, *nz; float *ar, *ag, *ab; int32_t* material;
    int32_t* cell; float* hit_logit; int32_t* n_queried; float *xr, *yr, *zr;
    float *dnx, *dny, *dnz;     /* the normal carried to deformed space: (dD/dx)^-T n at the
                                   rest hit point, normalized (for shading the posed surface) */
} nif_hits;
enum { NIF_Q_FIRST_HIT = 0, NIF_Q_NO_NETWORK = 8, NIF_Q_POSE_TIMES = 16, NIF_Q_POSE_ORDER = 32 };
/* flags: NIF_Q_FIRST_HIT, or NIF_Q_NO_NETWORK (the voxel proxy: first occupied voxel is
 * the hit, D = t_in, no network); NIF_Q_POSE_TIMES adds per-pose completion times;
 * NIF_Q_POSE_ORDER (first-hit query) deals the rays pose by pose: each of the 8 per-XCD ray
 * ranges walks its eighth of pose 0, then of pose 1, and so on, so that poses complete in
 * order rather than all near the end of the launch (per-ray results are the same).
 * precision: NIF_PREC_*.  stats_dev: nullable int64[4] {rays done, network evaluations,
 * degenerate voxel tests, reserved}, accumulated; with NIF_Q_POSE_TIMES it must hold
 * 5 + 2 n_poses entries: [4] the kernel's start and [5 + p] the completion of pose p, in
 * device wall-clock ticks (hipDeviceAttributeWallClockRate kHz), [5 + n_poses + p] rays of
 * pose p finished; these are reset by the call. */
int nif_query(const nif_model* model, const nif_grid* grid, const nif_rays* rays, int64_t n_rays,
              const nif_hits* out, uint32_t flags, int32_t precision, int64_t* stats_dev,
              nif_stream stream);
/* Frequency of the current device's wall clock (the ticks of NIF_Q_POSE_TIMES), in kHz. */
int nif_wall_clock_khz(int32_t* khz);
/* Launch shape of the fused query: persistent one-wave workgroups per compute unit,
 * 1..32 (default 12).  Process-wide. */
int nif_set_query_blocks_per_cu(int32_t blocks_per_cu);
/* Rays each wave of the fused query walks at a time: 64, or 16 (one network pass of 16
 * segments per round instead of four: shorter serial chains for launches too small to fill
 * the GPU), or 0 = chosen from the launch size (16 below 8192 rays per compute unit).
 * Process-wide; results do not depend on it. */
int nif_set_query_rays_per_wave(int32_t rays_per_wave);
/* Measurement support (not part of the method): device ceilings that the rooflines are read
 * against, each timed with device events over `reps` launches after one warm-up.
 *   NIF_MB_HBM_READ    streaming float4 reads of an n_bytes buffer: result[0] = bytes/s
 *   NIF_MB_GATHER4     n_ops random 4-byte gathers (one half2 table entry) at hashed indices of
 *                      an n_bytes table, eight in flight per lane: result[0] = gathered bytes/s
 *   NIF_MB_GATHER8     the same with 8-byte gathers (an aligned entry pair)
 *   NIF_MB_MFMA_F32    n_ops v_mfma_f32_16x16x4_f32 (four independent chains per wave): FLOP/s
 *   NIF_MB_MFMA_BF16   n_ops v_mfma_f32_16x16x16_bf16: FLOP/s
 * result[1] = milliseconds per launch.  Allocates and frees its buffers; synchronises the
 * stream.  n_bytes: a multiple of 16 in [4096, 2^33] (memory kinds); n_ops in [1, 2^40]. */
enum { NIF_MB_HBM_READ = 0, NIF_MB_GATHER4 = 1, NIF_MB_GATHER8 = 2, NIF_MB_MFMA_F32 = 3, NIF_MB_MFMA_BF16 = 4 };
int nif_microbench(int32_t kind, int64_t n_bytes, int64_t n_ops, int32_t reps, double* result, nif_stream stream);
/* Autotuner of the fused query's launch shape: runs nif_query on the caller's rays (flags 0,
 * no stats) once to warm up and `reps` times timed with device events, for every pair of
 * workgroups per CU in {4, 6, 8, 10, 12, 14, 16, 20, 24} and rays per wave in {16, 64}; keeps
 * the fastest pair process-wide (as the two setters above would) and returns it in
 * best[0] (workgroups per CU), best[1] (rays per wave), with its time per launch in
 * *best_ms (nullable).  Outputs are those of the last launch (they do not depend on the
 * shape).  Synchronises the stream; not for graph capture.  On an error the previous shape
 * is kept. */
int nif_autotune_query(const nif_model* model, const nif_grid* grid, const nif_rays* rays, int64_t n_rays,
                       const nif_hits* out, int32_t precision, int32_t reps, int32_t* best, float* best_ms,
                       nif_stream stream);

/* ---------------------------------------------------------------- network on points
 * Grid encoding of n rest-space points (SoA [3][n]) -> out[n][(1+2F) L feat_dim], FP32: psi;
 * with concat_encoding, phi of the points themselves, out[n][L feat_dim]. */
int nif_encode(const nif_model* model, const float* x_dev, int64_t n, float* out_dev, nif_stream stream);
/* Heads of B point pairs: heads_dev[B][8 + n_materials] = MLP(psi(x0) ++ psi(x1)). */
int nif_forward(const nif_model* model, const float* x0_dev, const float* x1_dev, int64_t B,
                float* heads_dev, int32_t precision, nif_stream stream);
/* Backward of nif_forward given d heads [B][8 + n_materials]: adds dL/dtables, dL/dmlp to
 * the model's gradient accumulators (zeroed first unless accumulate != 0) and writes
 * dL/dx0, dL/dx1 (SoA, nullable).  Hand-written: MLP backward, hash-grid scatter-add with
 * the trilinear weights (additions grouped by table slice and summed in 64-bit fixed
 * point), PE chain rule.  Nothing is kept from nif_forward: the hidden activations are
 * recomputed, and the encoding is recomputed per chunk of 2^17 samples. */
int nif_backward(nif_model* model, const float* x0_dev, const float* x1_dev, int64_t B,
                 const float* d_heads_dev, float* d_x0_dev, float* d_x1_dev, int32_t accumulate,
                 int32_t precision, nif_stream stream);

/* ---------------------------------------------------------------- training
 * One step of training on a batch of B voxel segments with rest-space supervision
 * (Methodology: a dataset of deformed-space ray queries with rest-space labels): forward,
 * uncertainty-weighted multi-task loss ("Uncertainty-Weighted Multi-Task Loss": regression
 * 0.5 e^-s L + 0.5 s for distance (log-space MSE, eps 1e-4), normal (1 - cos) and albedo
 * (L1 of sigmoid); classification e^-s L + 0.5 s for occlusion (BCE) and material (CE);
 * geometric and appearance terms averaged over the hit samples only), backward and Adam
 * (bias-corrected; lr for tables, MLP and s).  BF16/FP16 use dynamic loss scaling: a
 * non-finite gradient skips the update and halves the scale.
 * losses_dev: float[16] = {L_hit, L_dist, L_nrm, L_alb, L_mat, total, s[5], loss scale,
 * skipped (0/1), n_hit, 0, 0}. */
typedef struct {
    const float *x0, *x1;       /* SoA [3][B] rest-space entry / exit points */
    const uint8_t* hit;         /* [B] occlusion label */
    const float* t;             /* [B] rest-space distance from x0 along the segment */
    const float* n;             /* SoA [3][B] unit normal */
    const float* a;             /* SoA [3][B] albedo */
    const int32_t* m;           /* [B] material id */
} nif_batch;
typedef struct {
    float lr_table, lr_mlp, lr_s, beta1, beta2, eps;
    int32_t precision;          /* NIF_PREC_* of the MLP */
    float loss_scale_init;      /* 0 = 1 for FP32/BF16, 32768 for FP16 */
    int32_t fixed_task_weights; /* 1 = ablation without uncertainty weighting: total = sum of
                                   the five task losses, s neither used nor updated */
    int32_t store_encoding;     /* 0: the forward keeps no encoding; the backward recomputes it
                                   (gathers again) per chunk of 2^17 samples for the first
                                   layer's weight gradient, in a [2^17][E] FP32 scratch.
                                   1: the forward stores the [B][E] FP32 encoding for the
                                   backward (one gather pass less per step; max_batch E 4 bytes
                                   more device memory, from nif_model_reserve_encoding; without
                                   it the step fails with NIF_E_STATE).  The hidden activations
                                   are stored in both cases. */
    int32_t loss_scale_growth_interval; /* dynamic loss scaling (BF16/FP16): the scale doubles
                                   after this many clean steps in a row; 0 = 1000.  A step with
                                   a non-finite loss or gradient is skipped (no parameter,
                                   moment or step-counter change) and halves the scale (not
                                   below 2^-16).  FP32 steps keep the scale at 1. */
} nif_train_cfg;
int nif_train_step(nif_model* model, const nif_batch* batch, int64_t B, const nif_train_cfg* cfg,
                   float* losses_dev, nif_stream stream);

/* The training step's loss on its own ("Uncertainty-Weighted Multi-Task Loss"), for callers
 * that run the network themselves (the Python autograd wrapper): heads_dev [B][8 + n_materials]
 * are raw MLP outputs, labels as in nif_batch (x0 / x1 read only by the sigmoid distance head),
 * s_dev[5] the task log-variances.  Writes losses_dev[6] = {L_hit, L_dist, L_nrm, L_alb,
 * L_mat, total}, d_heads_dev [B][8 + n_materials] = d total / d heads (nullable) and
 * d_s_dev[5] = d total / d s (nullable; zero with fixed_task_weights, as in nif_train_cfg).
 * Uses the model's description and a few words of accumulator it owns (not those of the
 * training step); no allocation, no synchronisation. */
int nif_loss(nif_model* model, const float* heads_dev, int64_t B, const nif_batch* labels, const float* s_dev,
             int32_t fixed_task_weights, float* losses_dev, float* d_heads_dev, float* d_s_dev,
             nif_stream stream);

#ifdef __cplusplus
}
#endif
#endif
