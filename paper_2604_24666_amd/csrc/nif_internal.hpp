// Host-side state behind the opaque libnif handles, and the launchers each translation unit
// provides to the C ABI layer (nif_api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/nif.h"
#include "nif_device.hpp"

struct nif_grid {
    int32_t N = 0, n_poses = 0;
    std::vector<nif::PoseDev> poses_host;   // as last read back after the build
    nif::PoseDev* poses = nullptr;          // device [n_poses]
    float4* verts = nullptr;                // device [n_poses][(N+1)^3]
    int32_t* bin_start = nullptr;           // device, per pose nbins + 1 (exclusive scan)
    int32_t* bin_cells = nullptr;           // device, occupied voxel ids per bin
    int32_t* list = nullptr;                // device, occupied voxel ids (shared by all poses)
    int32_t* counts = nullptr;              // device, per-bin counters (build scratch)
    int32_t* scratch = nullptr;             // device, boxes / totals / flags
    int64_t* order_pre = nullptr;           // device [8][n_poses + 1]: pose-ordered dealing (query)
    int64_t bin_total = 0, max_bins = 0, ref_capacity = 0;
    int64_t n_occupied = 0;
    std::vector<int64_t> refs_per_pose;
};

struct nif_model {
    nif_model_desc desc{};
    int32_t S = 0;           // PE samples per point that go through the grid
    int32_t GW = 0;          // raw gamma values per point appended (concatenated encoding)
    int32_t E = 0;           // encoding width (both points)
    int32_t H = 0;           // head count (8 + materials)
    int64_t n_table = 0, n_mlp = 0;
    int32_t n_layers = 0;    // affine layers
    std::vector<int32_t> dims;          // [n_layers + 1], canonical (last = H)
    std::vector<int32_t> dims_pad;      // last padded to 16
    std::vector<int64_t> w_off, b_off;  // canonical offsets of each layer's W and b
    std::vector<int64_t> wp_off, bp_off;// offsets in the padded working copies
    std::vector<int64_t> wt_off;        // transposed padded copy of layer i: [in][out_pad]
    int64_t n_mlp_pad = 0;
    int64_t n_w0l = 0;                  // first-layer weights in the fused kernels' lane order
    float* w0l_f32 = nullptr;           //   [HW/16][U][L/4][2][64 lanes][4], U = ceil(2S/4)
    uint16_t* w0l_bf16 = nullptr;
    __half* w0l_f16 = nullptr;
    // parameters
    float* tables = nullptr;            // FP32 master [L][T][Fd]
    __half* tables_h = nullptr;         // FP16 working copy (table_dtype == F16)
    float* mlp = nullptr;               // FP32 master, canonical
    float* mlp_pad_f32 = nullptr;       // padded working copies
    uint16_t* mlp_pad_bf16 = nullptr;
    __half* mlp_pad_f16 = nullptr;
    float* s = nullptr;                 // [5]
    // gradients (FP32, canonical layout) and Adam moments
    float *g_tables = nullptr, *g_mlp = nullptr, *g_s = nullptr;
    float *m_tables = nullptr, *v_tables = nullptr, *m_mlp = nullptr, *v_mlp = nullptr;
    float *m_s = nullptr, *v_s = nullptr;
    // the backward runs the table-gradient chain on `side` beside the weight gradients
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // training scratch (sized for max_batch samples; grown only by nif_model_reserve)
    int64_t max_batch = 0;
    float* zbuf = nullptr;              // [max_batch][H] heads of the training forward
    float* dz = nullptr;                // [max_batch][16] d loss / d heads (loss-scaled, padded)
    float* acts = nullptr;              // [hidden_layers][max_batch][hidden_width] post-ReLU
    float* delta = nullptr;             // [hidden_layers][max_batch][hidden_width] d loss / d pre-activation
    float* enc = nullptr;               // [bwd_chunk][E] encoding recomputed for the first layer's dW
    float* enc_all = nullptr;           // [max_batch][E] stored encoding (store_encoding steps only;
                                        //   allocated by nif_model_reserve_encoding)
    int64_t bwd_chunk = 0;              // samples per training chunk (forward, MLP backward, one fill launch)
    int64_t bwd_round = 0;              // samples per table-gradient round (count, scan, reduce): whole chunks
    int32_t* bwd_cnt = nullptr;         // [buckets][blocks] addition counts / offsets
    int32_t* bwd_scan = nullptr;        // scan partial sums + total
    float* bwd_val = nullptr;           // table-gradient records, 16 bytes each (corner-pair records with two features)
    uint32_t* ord_u32 = nullptr;        // batch ordering: keys and indices, 2 x 2 x max_batch
    float* ord_f32 = nullptr;           //   the ordered batch (15 max_batch words)
    void* ord_temp = nullptr;           //   radix-sort scratch
    size_t ord_temp_bytes = 0;
    float* dw_part = nullptr;           // weight-gradient partial sums per K slice
    int64_t dw_part_n = 0;              //   capacity in floats
    double* dacc = nullptr;             // [16] loss sums, loss scale, Adam bias corrections
    int64_t* tcount = nullptr;          // [16] positives, step, clean steps, flags
    int32_t step = 0;
    bool params_set = false;
    int64_t* counters = nullptr;        // [8] query work counters
};

namespace nif {

// error reporting (thread-local message)
int fail(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

// nif_grid.hip
int grid_build(nif_grid* g, const uint8_t* occ, int32_t N, const nif_pose* poses, int32_t n_poses,
               int32_t bins_per_axis, hipStream_t st);
void grid_free(nif_grid* g);
int grid_update(nif_grid* g, const nif_pose* poses, hipStream_t st);
int grid_bounds(const nif_grid* g, int pose, float* lo, float* hi);
int grid_overflow(nif_grid* g, hipStream_t st, int32_t* overflow);
int voxelize_launch(int32_t scene_kind, const float* params_dev, int32_t N, uint8_t* occ,
                    hipStream_t st);

// nif_query.hip
int trace_launch(const nif_grid* g, const nif_rays* r, int64_t n, int32_t max_seg,
                 const nif_segments* out, hipStream_t st);
int query_launch(const nif_model* m, const nif_grid* g, const nif_rays* r, int64_t n,
                 const nif_hits* out, uint32_t flags, int32_t precision, int64_t* stats,
                 hipStream_t st);
int set_query_blocks_per_cu(int v);
int set_query_rays_per_wave(int v);
int autotune_query(const nif_model* m, const nif_grid* g, const nif_rays* r, int64_t n, const nif_hits* out,
                   int32_t precision, int32_t reps, int32_t* best, float* best_ms, hipStream_t st);
int encode_launch(const nif_model* m, const float* x, int64_t n, float* out, hipStream_t st);
int label_launch(int kind, const double* params_host, int32_t n_params, int force_march, const float* x0,
                 const float* x1, int64_t n, uint8_t* hit, float* t, float* nrm, float* alb, int32_t* mat,
                 hipStream_t st);
// Same labels with the scene parameters staged in a static per-device array (no allocation,
// no synchronisation); n_params <= kLabelScratchDoubles.
constexpr int32_t kLabelScratchDoubles = 4104;
int label_launch_noalloc(int kind, const double* params_host, int32_t n_params, int force_march, const float* x0,
                         const float* x1, int64_t n, uint8_t* hit, float* t, float* nrm, float* alb, int32_t* mat,
                         hipStream_t st);
int forward_launch(const nif_model* m, const float* x0, const float* x1, int64_t B, float* heads,
                   int32_t precision, float* acts, float* enc, hipStream_t st);
// Forward of n pairs whose SoA rows have stride ld (heads [n][H], acts [layers][n][HW] and enc
// [n][E] local to the n rows).
int forward_rows_launch(const nif_model* m, const float* x0, const float* x1, int64_t n, int64_t ld, float* heads,
                        int32_t precision, float* acts, float* enc, hipStream_t st);
// Encoding only of n pairs whose SoA rows have stride ld: enc[n][E], the values the forward
// of the same precision feeds its first layer.
int encode_pairs_launch(const nif_model* m, const float* x0, const float* x1, int64_t n, int64_t ld,
                        int32_t precision, float* enc, hipStream_t st);

// nif_train.hip
int model_alloc(nif_model* m);
void model_free(nif_model* m);
int model_sync_working(nif_model* m, hipStream_t st);
int model_sync_mlp(nif_model* m, hipStream_t st);
int zero_grads_launch(nif_model* m, hipStream_t st);
int microbench(int32_t kind, int64_t n_bytes, int64_t n_ops, int32_t reps, double* result, hipStream_t st);
int backward_launch(nif_model* m, const float* x0, const float* x1, int64_t B, const float* dh,
                    int32_t dh_stride, float* dx0, float* dx1, int32_t precision, hipStream_t st);
int train_step_launch(nif_model* m, const nif_batch* b, int64_t B, const nif_train_cfg* cfg,
                      float* losses, hipStream_t st);
int model_reserve(nif_model* m, int64_t B);
int model_reserve_encoding(nif_model* m);
int loss_launch(nif_model* m, const float* heads, int64_t B, const nif_batch* b, const float* s, int32_t fixed,
                float* losses, float* d_heads, float* d_s, hipStream_t st);

// nif_order.hip
size_t order_temp_bytes(int64_t B);
int order_batch(nif_model* m, const nif_batch* b, int64_t B, nif_batch* sorted, hipStream_t st);

}  // namespace nif
