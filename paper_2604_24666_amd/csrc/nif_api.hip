// C ABI of libnif: argument validation, handle management and dispatch to the launchers.
// Every argument error is caught here, before anything is enqueued.
#include <cstdio>
#include <cstring>
#include <string>

#include "nif_internal.hpp"

namespace nif {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return NIF_OK;
    return fail(NIF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace nif

using nif::fail;

#define REQUIRE(cond, msg)                                  \
    do {                                                    \
        if (!(cond)) return fail(NIF_E_INVALID_ARG, (msg)); \
    } while (0)

static hipStream_t S(nif_stream s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" {

const char* nif_status_string(int status) {
    switch (status) {
        case NIF_OK: return "ok";
        case NIF_E_INVALID_ARG: return "invalid argument";
        case NIF_E_UNSUPPORTED: return "unsupported";
        case NIF_E_OOM: return "out of device memory";
        case NIF_E_DEVICE: return "device error";
        case NIF_E_STATE: return "invalid state";
        default: return "unknown status";
    }
}

const char* nif_last_error(void) { return nif::g_last_error.c_str(); }

int nif_version(void) { return 1; }

static int validate_desc(const nif_model_desc* d) {
    REQUIRE(d, "desc is null");
    REQUIRE(d->feat_dim == 2 || d->feat_dim == 3, "feat_dim must be 2 or 3");
    if (d->feat_dim == 2) REQUIRE(d->levels == 4 || d->levels == 8 || d->levels == 12 || d->levels == 16,
                                  "with feat_dim 2, levels must be 4, 8, 12 or 16");
    else REQUIRE(d->levels >= 2 && d->levels <= 16 && d->levels % 2 == 0, "with feat_dim 3, levels must be even in [2, 16]");
    REQUIRE(d->feat_dim == 2 || d->concat_encoding == 0, "the concatenated encoding needs feat_dim 2");
    REQUIRE(d->log2_table >= 4 && d->log2_table <= 24, "log2_table must be in [4, 24]");
    REQUIRE(d->table_dtype == NIF_TABLE_F32 || d->table_dtype == NIF_TABLE_F16, "table_dtype must be NIF_TABLE_F32 or NIF_TABLE_F16");
    for (int l = 0; l < d->levels; ++l) REQUIRE(d->res[l] >= 1 && d->res[l] <= (1 << 20), "res[l] must be in [1, 2^20]");
    REQUIRE(d->pe_freqs >= 0 && d->pe_freqs <= 12, "pe_freqs must be in [0, 12]");
    if (!(d->hidden_width == 16 || d->hidden_width == 32 || d->hidden_width == 64 || d->hidden_width == 128))
        return fail(NIF_E_UNSUPPORTED, "hidden_width must be 16, 32, 64 or 128");
    REQUIRE(d->hidden_layers >= 1 && d->hidden_layers <= 8, "hidden_layers must be in [1, 8]");
    REQUIRE(d->n_materials >= 1 && d->n_materials <= 8, "n_materials must be in [1, 8]");
    REQUIRE(d->dist_head == NIF_DIST_LOG_RELU || d->dist_head == NIF_DIST_SIGMOID,
            "dist_head must be NIF_DIST_LOG_RELU or NIF_DIST_SIGMOID");
    REQUIRE(d->per_sample_tables == 0 || d->per_sample_tables == 1, "per_sample_tables must be 0 or 1");
    REQUIRE(d->concat_encoding == 0 || d->concat_encoding == 1, "concat_encoding must be 0 or 1");
    REQUIRE((d->per_sample_tables ? (int64_t)(d->concat_encoding ? 1 : 1 + 2 * d->pe_freqs) : 1) * d->levels
                    * ((int64_t)1 << d->log2_table) < ((int64_t)1 << 32),
            "the tables must hold fewer than 2^32 entries");
    return NIF_OK;
}

int nif_model_sizes(const nif_model_desc* d, int64_t* n_table, int64_t* n_mlp) {
    int rc = validate_desc(d);
    if (rc) return rc;
    const int64_t Sg = d->concat_encoding ? 1 : 1 + 2 * d->pe_freqs;
    const int64_t E = 2LL * (Sg * d->levels * d->feat_dim + (d->concat_encoding ? 3 * (1 + 2 * d->pe_freqs) : 0));
    const int64_t H = 8 + d->n_materials;
    int64_t n = 0, prev = E;
    for (int i = 0; i < d->hidden_layers; ++i) { n += (int64_t)d->hidden_width * prev + d->hidden_width; prev = d->hidden_width; }
    n += H * prev + H;
    if (n_table) *n_table = (int64_t)(d->per_sample_tables ? Sg : 1) * d->levels *
                            ((int64_t)1 << d->log2_table) * d->feat_dim;
    if (n_mlp) *n_mlp = n;
    return NIF_OK;
}

int nif_model_create(const nif_model_desc* desc, nif_model** out) {
    int rc = validate_desc(desc);
    if (rc) return rc;
    REQUIRE(out, "out is null");
    nif_model* m = new nif_model();
    m->desc = *desc;
    rc = nif::model_alloc(m);
    if (rc) {
        nif::model_free(m);
        delete m;
        return rc;
    }
    *out = m;
    return NIF_OK;
}

int nif_model_destroy(nif_model* m) {
    if (!m) return NIF_OK;
    nif::model_free(m);
    delete m;
    return NIF_OK;
}

int nif_model_set_params(nif_model* m, const float* tables, const float* mlp, const float* s, nif_stream stream) {
    REQUIRE(m, "model is null");
    REQUIRE(tables && mlp, "tables and mlp must not be null");
    hipStream_t st = S(stream);
    int rc;
    if ((rc = nif::check_hip(hipMemcpyAsync(m->tables, tables, sizeof(float) * m->n_table, hipMemcpyDeviceToDevice, st), "copy tables"))) return rc;
    if ((rc = nif::check_hip(hipMemcpyAsync(m->mlp, mlp, sizeof(float) * m->n_mlp, hipMemcpyDeviceToDevice, st), "copy mlp"))) return rc;
    if (s) {
        if ((rc = nif::check_hip(hipMemcpyAsync(m->s, s, sizeof(float) * 5, hipMemcpyDeviceToDevice, st), "copy s"))) return rc;
    } else if ((rc = nif::check_hip(hipMemsetAsync(m->s, 0, sizeof(float) * 8, st), "zero s"))) {
        return rc;
    }
    const struct { void* p; int64_t n; } zs[] = {{m->g_tables, m->n_table}, {m->g_mlp, m->n_mlp},
                                                 {m->g_s, 8}, {m->m_tables, m->n_table}, {m->v_tables, m->n_table},
                                                 {m->m_mlp, m->n_mlp}, {m->v_mlp, m->n_mlp}, {m->m_s, 8}, {m->v_s, 8}};
    for (auto& z : zs)
        if ((rc = nif::check_hip(hipMemsetAsync(z.p, 0, sizeof(float) * z.n, st), "zero state"))) return rc;
    if ((rc = nif::model_sync_working(m, st))) return rc;
    if ((rc = nif::check_hip(hipMemsetAsync(m->dacc, 0, sizeof(double) * 16, st), "zero train state"))) return rc;
    if ((rc = nif::check_hip(hipMemsetAsync(m->tcount, 0, sizeof(int64_t) * 16, st), "zero train state"))) return rc;
    m->step = 0;
    m->params_set = true;
    return NIF_OK;
}

int nif_model_get_params(const nif_model* m, float* tables, float* mlp, float* s, nif_stream stream) {
    REQUIRE(m, "model is null");
    hipStream_t st = S(stream);
    int rc;
    if (tables && (rc = nif::check_hip(hipMemcpyAsync(tables, m->tables, sizeof(float) * m->n_table, hipMemcpyDeviceToDevice, st), "copy tables"))) return rc;
    if (mlp && (rc = nif::check_hip(hipMemcpyAsync(mlp, m->mlp, sizeof(float) * m->n_mlp, hipMemcpyDeviceToDevice, st), "copy mlp"))) return rc;
    if (s && (rc = nif::check_hip(hipMemcpyAsync(s, m->s, sizeof(float) * 5, hipMemcpyDeviceToDevice, st), "copy s"))) return rc;
    return NIF_OK;
}

int nif_model_get_grads(const nif_model* m, float* gt, float* gm, float* gs, nif_stream stream) {
    REQUIRE(m, "model is null");
    hipStream_t st = S(stream);
    int rc;
    if (gt && (rc = nif::check_hip(hipMemcpyAsync(gt, m->g_tables, sizeof(float) * m->n_table, hipMemcpyDeviceToDevice, st), "copy grads"))) return rc;
    if (gm && (rc = nif::check_hip(hipMemcpyAsync(gm, m->g_mlp, sizeof(float) * m->n_mlp, hipMemcpyDeviceToDevice, st), "copy grads"))) return rc;
    if (gs && (rc = nif::check_hip(hipMemcpyAsync(gs, m->g_s, sizeof(float) * 5, hipMemcpyDeviceToDevice, st), "copy grads"))) return rc;
    return NIF_OK;
}

int nif_model_zero_grads(nif_model* m, nif_stream stream) {
    REQUIRE(m, "model is null");
    return nif::zero_grads_launch(m, S(stream));
}

int nif_model_reserve(nif_model* m, int64_t max_batch) {
    REQUIRE(m, "model is null");
    REQUIRE(max_batch >= 0 && max_batch <= (1LL << 26), "max_batch must be in [0, 2^26]");
    return nif::model_reserve(m, max_batch);
}

int nif_model_reserve_encoding(nif_model* m) {
    REQUIRE(m, "model is null");
    return nif::model_reserve_encoding(m);
}

int nif_voxelize(int32_t kind, const double* params, int32_t n_params, int32_t N, uint8_t* occ, nif_stream stream) {
    REQUIRE(kind >= 0 && kind <= 2, "scene_kind must be 0 (torus), 1 (spheres) or 2 (blobs)");
    REQUIRE(params && n_params >= 1, "params must not be empty");
    REQUIRE(N >= 1 && N <= 1024, "N must be in [1, 1024]");
    REQUIRE(occ, "occ is null");
    if (kind == 0) REQUIRE(n_params >= 5, "torus needs 5 parameters");
    else REQUIRE(params[0] >= 0 && n_params >= 1 + 8 * (int64_t)params[0], "parameter count does not match n");
    std::vector<float> pf(params, params + n_params);
    float* dp = nullptr;
    hipStream_t st = S(stream);
    int rc;
    if ((rc = nif::check_hip(hipMalloc(&dp, sizeof(float) * n_params), "hipMalloc scene"))) return rc;
    rc = nif::check_hip(hipMemcpyAsync(dp, pf.data(), sizeof(float) * n_params, hipMemcpyHostToDevice, st), "copy scene");
    if (!rc) rc = nif::voxelize_launch(kind, dp, N, occ, st);
    if (!rc) rc = nif::check_hip(hipStreamSynchronize(st), "voxelize sync");
    (void)hipFree(dp);
    return rc;
}

int nif_label(int32_t kind, const double* params, int32_t n_params, int32_t force_march, const float* x0,
              const float* x1, int64_t n, uint8_t* hit, float* t, float* nrm, float* alb, int32_t* mat,
              nif_stream stream) {
    REQUIRE(kind >= 0 && kind <= 2, "scene_kind must be 0 (torus), 1 (spheres) or 2 (blobs)");
    REQUIRE(params && n_params >= 1, "params must not be empty");
    if (kind == 0) REQUIRE(n_params >= 5, "torus needs 5 parameters");
    else REQUIRE(params[0] >= 0 && n_params >= 1 + 8 * (int64_t)params[0], "parameter count does not match n");
    REQUIRE(n >= 0, "n must be >= 0");
    if (n > 0) REQUIRE(x0 && x1, "x0 and x1 must not be null");
    return nif::label_launch(kind, params, n_params, force_march, x0, x1, n, hit, t, nrm, alb, mat, S(stream));
}

static_assert(NIF_LABEL_NOALLOC_MAX_PARAMS == nif::kLabelScratchDoubles, "label scratch size");

int nif_label_noalloc(int32_t kind, const double* params, int32_t n_params, int32_t force_march, const float* x0,
                      const float* x1, int64_t n, uint8_t* hit, float* t, float* nrm, float* alb, int32_t* mat,
                      nif_stream stream) {
    REQUIRE(kind >= 0 && kind <= 2, "scene_kind must be 0 (torus), 1 (spheres) or 2 (blobs)");
    REQUIRE(params && n_params >= 1, "params must not be empty");
    REQUIRE(n_params <= NIF_LABEL_NOALLOC_MAX_PARAMS, "n_params exceeds NIF_LABEL_NOALLOC_MAX_PARAMS (4104)");
    if (kind == 0) REQUIRE(n_params >= 5, "torus needs 5 parameters");
    else REQUIRE(params[0] >= 0 && n_params >= 1 + 8 * (int64_t)params[0], "parameter count does not match n");
    REQUIRE(n >= 0, "n must be >= 0");
    if (n > 0) REQUIRE(x0 && x1, "x0 and x1 must not be null");
    return nif::label_launch_noalloc(kind, params, n_params, force_march, x0, x1, n, hit, t, nrm, alb, mat, S(stream));
}

int nif_build_grid(const uint8_t* occ, int32_t N, const nif_pose* poses, int32_t n_poses, int32_t bins_per_axis,
                   nif_grid** out, nif_stream stream) {
    REQUIRE(occ, "occ is null");
    REQUIRE(N >= 1 && N <= 1024, "N must be in [1, 1024]");
    REQUIRE(poses && n_poses >= 1 && n_poses <= 4096, "n_poses must be in [1, 4096]");
    REQUIRE(bins_per_axis >= 0 && bins_per_axis <= 4096, "bins_per_axis must be in [0, 4096]");
    REQUIRE(out, "out is null");
    for (int p = 0; p < n_poses; ++p) {
        REQUIRE(poses[p].kind >= 0 && poses[p].kind <= 4, "unknown deformation kind");
        REQUIRE(poses[p].strength >= 0.f && poses[p].strength <= 1.f, "pose strength must be in [0, 1]");
    }
    nif_grid* g = new nif_grid();
    int rc = nif::grid_build(g, occ, N, poses, n_poses, bins_per_axis, S(stream));
    if (rc) {
        nif::grid_free(g);
        delete g;
        return rc;
    }
    *out = g;
    return NIF_OK;
}

int nif_grid_destroy(nif_grid* g) {
    if (!g) return NIF_OK;
    nif::grid_free(g);
    delete g;
    return NIF_OK;
}

int nif_grid_update(nif_grid* g, const nif_pose* poses, int32_t n_poses, nif_stream stream) {
    REQUIRE(g, "grid is null");
    REQUIRE(poses && n_poses == g->n_poses, "n_poses must equal the grid's pose count");
    for (int p = 0; p < n_poses; ++p) {
        REQUIRE(poses[p].kind >= 0 && poses[p].kind <= 4, "unknown deformation kind");
        REQUIRE(poses[p].strength >= 0.f && poses[p].strength <= 1.f, "pose strength must be in [0, 1]");
    }
    return nif::grid_update(g, poses, S(stream));
}

int nif_grid_info(const nif_grid* g, int32_t pose, int64_t* n_occupied, int64_t* n_refs, int32_t* overflow) {
    REQUIRE(g, "grid is null");
    REQUIRE(pose >= 0 && pose < g->n_poses, "pose out of range");
    if (n_occupied) *n_occupied = g->n_occupied;
    if (n_refs) *n_refs = g->refs_per_pose[pose];
    if (overflow) return nif::grid_overflow(const_cast<nif_grid*>(g), nullptr, overflow);
    return NIF_OK;
}

int nif_grid_bounds(const nif_grid* g, int32_t pose, float* lo, float* hi) {
    REQUIRE(g, "grid is null");
    REQUIRE(pose >= 0 && pose < g->n_poses, "pose out of range");
    REQUIRE(lo && hi, "lo and hi must not be null");
    return nif::grid_bounds(g, pose, lo, hi);
}

static int validate_rays(const nif_rays* r, int64_t n) {
    REQUIRE(r, "rays is null");
    REQUIRE(n >= 0, "n_rays must be >= 0");
    if (n > 0) REQUIRE(r->ox && r->oy && r->oz && r->dx && r->dy && r->dz && r->pose_offsets, "ray arrays must not be null");
    return NIF_OK;
}

int nif_trace(const nif_grid* g, const nif_rays* rays, int64_t n, int32_t max_seg, const nif_segments* out, nif_stream stream) {
    REQUIRE(g, "grid is null");
    int rc = validate_rays(rays, n);
    if (rc) return rc;
    REQUIRE(out, "out is null");
    REQUIRE(max_seg >= 0, "max_seg must be >= 0");
    if (n > 0) REQUIRE(out->count, "out->count must not be null");
    return nif::trace_launch(g, rays, n, max_seg, out, S(stream));
}

int nif_query(const nif_model* m, const nif_grid* g, const nif_rays* rays, int64_t n, const nif_hits* out, uint32_t flags,
              int32_t precision, int64_t* stats, nif_stream stream) {
    REQUIRE(g, "grid is null");
    int rc = validate_rays(rays, n);
    if (rc) return rc;
    REQUIRE(out, "out is null");
    REQUIRE((flags & ~(uint32_t)(NIF_Q_NO_NETWORK | NIF_Q_POSE_TIMES | NIF_Q_POSE_ORDER)) == 0, "unknown query flags");
    REQUIRE(precision >= 0 && precision <= 2, "precision must be NIF_PREC_FP32, _BF16 or _FP16");
    if (!(flags & NIF_Q_NO_NETWORK)) {
        REQUIRE(m, "model is null");
        if (!m->params_set) return fail(NIF_E_STATE, "model parameters were never set");
    }
    return nif::query_launch(m, g, rays, n, out, flags, precision, stats, S(stream));
}

int nif_wall_clock_khz(int32_t* khz) {
    REQUIRE(khz, "khz is null");
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess || v <= 0)
        return fail(NIF_E_DEVICE, "wall clock rate not available");
    *khz = v;
    return NIF_OK;
}

int nif_set_query_blocks_per_cu(int32_t v) {
    REQUIRE(v >= 1 && v <= 32, "blocks_per_cu must be in [1, 32]");
    return nif::set_query_blocks_per_cu(v);
}

int nif_microbench(int32_t kind, int64_t n_bytes, int64_t n_ops, int32_t reps, double* result, nif_stream stream) {
    REQUIRE(kind >= NIF_MB_HBM_READ && kind <= NIF_MB_MFMA_BF16, "kind must be one of NIF_MB_*");
    REQUIRE(result, "result is null");
    REQUIRE(reps >= 1 && reps <= 1000, "reps must be in [1, 1000]");
    REQUIRE(n_ops >= 1 && n_ops <= ((int64_t)1 << 40), "n_ops must be in [1, 2^40]");
    if (kind <= NIF_MB_GATHER8)
        REQUIRE(n_bytes >= 4096 && n_bytes % 16 == 0 && n_bytes <= ((int64_t)1 << 33),
                "n_bytes must be a multiple of 16 in [4096, 2^33]");
    return nif::microbench(kind, n_bytes, n_ops, reps, result, S(stream));
}

int nif_autotune_query(const nif_model* m, const nif_grid* g, const nif_rays* rays, int64_t n, const nif_hits* out,
                       int32_t precision, int32_t reps, int32_t* best, float* best_ms, nif_stream stream) {
    REQUIRE(g && m, "model and grid must not be null");
    int rc = validate_rays(rays, n);
    if (rc) return rc;
    REQUIRE(out && best, "out and best must not be null");
    REQUIRE(n >= 1, "n_rays must be >= 1");
    REQUIRE(precision >= 0 && precision <= 2, "precision must be NIF_PREC_FP32, _BF16 or _FP16");
    REQUIRE(reps >= 1 && reps <= 100, "reps must be in [1, 100]");
    if (!m->params_set) return fail(NIF_E_STATE, "model parameters were never set");
    return nif::autotune_query(m, g, rays, n, out, precision, reps, best, best_ms, S(stream));
}

int nif_set_query_rays_per_wave(int32_t v) {
    REQUIRE(v == 0 || v == 16 || v == 64, "rays_per_wave must be 0, 16 or 64");
    return nif::set_query_rays_per_wave(v);
}

int nif_encode(const nif_model* m, const float* x, int64_t n, float* out, nif_stream stream) {
    REQUIRE(m, "model is null");
    REQUIRE(n >= 0, "n must be >= 0");
    if (n > 0) REQUIRE(x && out, "x and out must not be null");
    if (!m->params_set) return fail(NIF_E_STATE, "model parameters were never set");
    return nif::encode_launch(m, x, n, out, S(stream));
}

int nif_forward(const nif_model* m, const float* x0, const float* x1, int64_t B, float* heads, int32_t precision,
                nif_stream stream) {
    REQUIRE(m, "model is null");
    REQUIRE(B >= 0, "B must be >= 0");
    if (B > 0) REQUIRE(x0 && x1 && heads, "x0, x1 and heads must not be null");
    REQUIRE(precision >= 0 && precision <= 2, "precision must be NIF_PREC_FP32, _BF16 or _FP16");
    if (!m->params_set) return fail(NIF_E_STATE, "model parameters were never set");
    return nif::forward_launch(m, x0, x1, B, heads, precision, nullptr, nullptr, S(stream));
}

int nif_backward(nif_model* m, const float* x0, const float* x1, int64_t B, const float* dh, float* dx0, float* dx1,
                 int32_t accumulate, int32_t precision, nif_stream stream) {
    REQUIRE(m, "model is null");
    REQUIRE(B >= 0, "B must be >= 0");
    if (B > 0) REQUIRE(x0 && x1 && dh, "x0, x1 and d_heads must not be null");
    REQUIRE(precision >= 0 && precision <= 2, "precision must be NIF_PREC_FP32, _BF16 or _FP16");
    if (!m->params_set) return fail(NIF_E_STATE, "model parameters were never set");
    if (B > m->max_batch) return fail(NIF_E_STATE, "batch larger than reserved with nif_model_reserve");
    int rc;
    if (!accumulate && (rc = nif_model_zero_grads(m, stream))) return rc;
    return nif::backward_launch(m, x0, x1, B, dh, m->H, dx0, dx1, precision, S(stream));
}

int nif_loss(nif_model* m, const float* heads, int64_t B, const nif_batch* labels, const float* s,
             int32_t fixed_task_weights, float* losses, float* d_heads, float* d_s, nif_stream stream) {
    REQUIRE(m, "model is null");
    REQUIRE(heads && labels && s && losses, "heads, labels, s and losses must not be null");
    REQUIRE(B >= 1, "B must be >= 1");
    REQUIRE(labels->hit && labels->t && labels->n && labels->a && labels->m, "label arrays must not be null");
    REQUIRE(fixed_task_weights == 0 || fixed_task_weights == 1, "fixed_task_weights must be 0 or 1");
    REQUIRE(m->desc.dist_head != NIF_DIST_SIGMOID || (labels->x0 && labels->x1),
            "the sigmoid distance head needs the segment end points x0, x1");
    return nif::loss_launch(m, heads, B, labels, s, fixed_task_weights, losses, d_heads, d_s, S(stream));
}

int nif_train_step(nif_model* m, const nif_batch* b, int64_t B, const nif_train_cfg* cfg, float* losses, nif_stream stream) {
    REQUIRE(m, "model is null");
    REQUIRE(b && cfg && losses, "batch, cfg and losses must not be null");
    REQUIRE(B >= 1, "B must be >= 1");
    REQUIRE(b->x0 && b->x1 && b->hit && b->t && b->n && b->a && b->m, "batch arrays must not be null");
    REQUIRE(cfg->precision >= 0 && cfg->precision <= 2, "precision must be NIF_PREC_FP32, _BF16 or _FP16");
    REQUIRE(cfg->beta1 >= 0.f && cfg->beta1 < 1.f && cfg->beta2 >= 0.f && cfg->beta2 < 1.f && cfg->eps > 0.f, "bad Adam hyper-parameters");
    REQUIRE(cfg->fixed_task_weights == 0 || cfg->fixed_task_weights == 1, "fixed_task_weights must be 0 or 1");
    REQUIRE(cfg->store_encoding == 0 || cfg->store_encoding == 1, "store_encoding must be 0 or 1");
    REQUIRE(cfg->loss_scale_growth_interval >= 0, "loss_scale_growth_interval must be >= 0");
    REQUIRE(cfg->loss_scale_init >= 0.f && cfg->loss_scale_init < 3.0e38f, "loss_scale_init must be finite and >= 0");
    if (!m->params_set) return fail(NIF_E_STATE, "model parameters were never set");
    if (B > m->max_batch) return fail(NIF_E_STATE, "batch larger than reserved with nif_model_reserve");
    return nif::train_step_launch(m, b, B, cfg, losses, S(stream));
}

}  // extern "C"
