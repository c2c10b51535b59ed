// Training step: uncertainty-weighted multi-task loss, hand-written backward and Adam.
//
// "Uncertainty-Weighted Multi-Task Loss": each task i has a learnable s_i = log sigma_i^2;
// regression tasks (distance as MSE of logs with a ReLU output, normal as 1 - cosine,
// albedo as L1 of sigmoid outputs) weigh 0.5 exp(-s) L + 0.5 s, classification tasks
// (occlusion, material; cross-entropy) exp(-s) L + 0.5 s.  Reading used here: occlusion is
// averaged over the whole batch, the geometric and appearance terms over the samples whose
// label is a hit; the distance epsilon is 1e-4.  The optimizer (Adam with bias correction)
// is not named by the paper.
//
// Launch sequence of one step (all on the caller's stream, no host synchronisation):
//   begin / count positives -> zero gradients -> forward (stores hidden activations) ->
//   loss and d loss / d heads (loss-scaled) -> MLP backward on MFMA (transposed weights,
//   deltas chained in registers) -> split-K dW GEMMs on MFMA -> encoding backward (the
//   encoding is recomputed chunk by chunk, d enc = W0^T delta, the table-gradient additions
//   with the trilinear weights grouped by table slice and summed in LDS, dW0) -> non-finite
//   check -> finalize
//   (losses, d/ds, dynamic loss scale) -> Adam on all parameters (FP16 table copy refreshed
//   in place) -> refresh of the MLP working copies.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "nif_internal.hpp"
#include "nif_net.hpp"

namespace nif {

NetParams make_net_params(const nif_model* m, int32_t precision);

enum { TC_NPOS = 0, TC_STEP = 1, TC_GOOD = 2, TC_NONFINITE = 3, TC_SKIP = 4 };
enum { DA_SUM = 0, DA_SCALE = 5, DA_SCALE_USED = 6, DA_C1 = 7, DA_C2 = 8 };
constexpr float kDistEps = 1e-4f;
constexpr int kGrowIntervalDefault = 1000;  // clean steps before the loss scale doubles
constexpr int64_t kEncBwdChunk = 1 << 17;  // samples per training chunk (and per fill launch)
constexpr int kEncBwdRoundChunks = 2;      // chunks per table-gradient round (count, scan, reduce)
constexpr int kBwdTilesPerBlock = 8;       // 16-sample tiles per encoding-backward block (4 waves)
constexpr int kRecFloats = 4;              // floats per table-gradient record (16 bytes)

// Concatenated encoding: d x of the appended gamma values, d enc_v = (W0^T delta_0)_v times
// d gamma_v / d x_a of the clamped coordinate (zero outside the cube), added to dx0 / dx1.
__global__ void __launch_bounds__(256) k_gamma_dx(const float* __restrict__ W0t, const float* __restrict__ delta0,
                                                  int HW, int E_phi, int GW, const float* __restrict__ x0,
                                                  const float* __restrict__ x1, int64_t B, float* __restrict__ dx0,
                                                  float* __restrict__ dx1) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < B; i += (int64_t)gridDim.x * blockDim.x) {
        const float* d = delta0 + i * HW;
        for (int p = 0; p < 2; ++p) {
            const float* xs = p ? x1 : x0;
            float* dx = p ? dx1 : dx0;
            float acc[3] = {0.f, 0.f, 0.f};
            for (int r = 0; r < GW; ++r) {
                const int s = r / 3, a = r - 3 * s;
                const float* w = W0t + (size_t)(E_phi + p * GW + r) * HW;
                float de = 0.f;
                for (int o = 0; o < HW; ++o) de = fmaf(w[o], d[o], de);
                const float x = fminf(fmaxf(xs[a * B + i], 0.f), 1.f);
                float dg = 1.f;
                if (s > 0) {
                    const float f = (float)(1 << ((s - 1) >> 1));
                    dg = (s - 1) & 1 ? -f * sinf(f * x) : f * cosf(f * x);
                }
                acc[a] = fmaf(de, dg, acc[a]);
            }
            for (int a = 0; a < 3; ++a) {
                const float xv = xs[a * B + i];
                if (xv >= 0.f && xv <= 1.f) dx[a * B + i] += acc[a];
            }
        }
    }
}

// Arguments of the weight-gradient kernels (k_dw_part, k_dw_sum).
struct DwArgs {
    const float* d; int dstride; int M_pad; int M_real;
    const float* h; int hstride; int N;
    int64_t B, Kc;
    int n_cb, ks;                // column tiles of 64, K slices per chunk
    float* part;                 // [slot][M_pad][N] then [slot][M_pad] bias sums
    int64_t n_slots;
};

constexpr int64_t kDwMinK = 512;
constexpr int kDwKT = 16;                  // samples per LDS-staged tile of k_dw_tile

// Launch shape of one layer's weight gradient: about two blocks per compute unit, each over at
// least kDwMinK samples.
static DwArgs dw_shape(int M_pad, int N, int64_t B, int cus) {
    DwArgs A;
    memset(&A, 0, sizeof(A));
    A.M_pad = M_pad; A.N = N; A.B = B;
    A.n_cb = (N + 63) / 64;
    A.ks = A.n_cb >= 4 ? 1 : 4 / A.n_cb;
    const int n_cg = (A.n_cb + 3) / 4;
    const int64_t target = 2LL * cus;
    int64_t nch = std::max<int64_t>(1, (target + n_cg - 1) / n_cg);
    // at least kDwMinK samples per K chunk: fewer partial slots for k_dw_sum to add up, and
    // each wave's MFMA loop long enough to cover its operand loads
    A.Kc = std::max<int64_t>(kDwMinK, (((B + nch - 1) / nch) + 15) / 16 * 16);
    nch = (B + A.Kc - 1) / A.Kc;
    A.n_slots = nch * A.ks;
    return A;
}

static int64_t dw_part_floats(const DwArgs& A) { return A.n_slots * A.M_pad * ((int64_t)A.N + 1); }

// The LDS-staged form (k_dw_tile) serves layers with 64 or 128 output rows and N % 4 == 0.
static bool dw_tiled(int M_pad, int N) { return (M_pad == 64 || M_pad == 128) && N % 4 == 0; }
// Column tiles per block of k_dw_tile: 4 waves per block, 64-row halves across them.
static int dw_tile_ct(int M_pad) { return M_pad == 128 ? 2 : 4; }

// Launch shape of k_dw_tile: about two blocks per compute unit, each over at least kDwTileMinK
// samples (the partial slots cost a write and a read of M_pad N floats each).
constexpr int64_t kDwTileMinK = 256;
static DwArgs dw_tile_shape(int M_pad, int N, int64_t B, int cus) {
    DwArgs A;
    memset(&A, 0, sizeof(A));
    A.M_pad = M_pad; A.N = N; A.B = B;
    A.n_cb = (N + 63) / 64;
    A.ks = 1;
    const int ct = dw_tile_ct(M_pad), n_cg = (A.n_cb + ct - 1) / ct;
    const int64_t nch = std::max<int64_t>(1, (2LL * cus + n_cg - 1) / n_cg);
    A.Kc = std::max<int64_t>(kDwTileMinK, (((B + nch - 1) / nch) + kDwKT - 1) / kDwKT * kDwKT);
    A.n_slots = (B + A.Kc - 1) / A.Kc;
    return A;
}

// Partial-slot floats any batch size can need for one layer: dw_shape never uses more K chunks
// than its first estimate ceil(2 cus / column groups).
static int64_t dw_part_floats_max(int M_pad, int N, int cus) {
    const int n_cb = (N + 63) / 64, ks = n_cb >= 4 ? 1 : 4 / n_cb, n_cg = (n_cb + 3) / 4;
    const int64_t nch = std::max<int64_t>(1, (2LL * cus + n_cg - 1) / n_cg);
    int64_t need = nch * ks * M_pad * ((int64_t)N + 1);
    if (dw_tiled(M_pad, N)) {             // k_dw_tile: slots <= ceil(2 cus / column groups) + 1
        const int ct = dw_tile_ct(M_pad), n_cgt = (n_cb + ct - 1) / ct;
        const int64_t slots = (2LL * cus + n_cgt - 1) / n_cgt + 1;
        need = std::max(need, slots * M_pad * ((int64_t)N + 1));
    }
    return need;
}

int model_reserve(nif_model* m, int64_t B) {
    if (B <= m->max_batch) return NIF_OK;
    for (float** p : {&m->zbuf, &m->dz, &m->acts, &m->delta, &m->enc, &m->enc_all})
        if (*p) { (void)hipFree(*p); *p = nullptr; }
    for (void** p : {(void**)&m->bwd_cnt, (void**)&m->bwd_scan, (void**)&m->bwd_val})
        if (*p) { (void)hipFree(*p); *p = nullptr; }
    m->max_batch = 0;
    {
        // encoding-backward additions: per chunk of samples, one per (sample, PE chunk, level, corner)
        const int log2T = m->desc.log2_table, L = m->desc.levels;
        const int SB = log2T <= 12 ? log2T : std::max(12, log2T - 8);
        const int64_t n_buckets = (int64_t)L * (m->desc.per_sample_tables ? m->S : 1) * (1 << (log2T - SB));
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(B, kEncBwdChunk));
        // a round's additions are indexed by int32 offsets
        const int64_t per = 2 * (int64_t)m->S * L * 8;
        int64_t round = std::min<int64_t>(std::max<int64_t>(B, 1), chunk * kEncBwdRoundChunks);
        while (round > chunk && round * per > INT32_MAX) round -= chunk;
        const int64_t n_blk = ((round + 15) / 16 + kBwdTilesPerBlock - 1) / kBwdTilesPerBlock;
        const int64_t n_add = round * per;
        const int64_t n_cnt = n_buckets * n_blk;
        const size_t sz[3] = {sizeof(int32_t) * (size_t)n_cnt,
                              sizeof(int32_t) * (size_t)((n_cnt + 4095) / 4096 + 3 + n_buckets),
                              // the reduction reads whole aligned groups of 16 records
                              sizeof(float) * kRecFloats * (size_t)(n_add + 16)};
        void** ptr[3] = {(void**)&m->bwd_cnt, (void**)&m->bwd_scan, (void**)&m->bwd_val};
        for (int i = 0; i < 3; ++i)
            if (hipMalloc(ptr[i], sz[i]) != hipSuccess) {
                (void)hipGetLastError();
                return fail(NIF_E_OOM, "encoding-backward buffer allocation failed");
            }
        m->bwd_chunk = chunk;
        m->bwd_round = round;
    }
    const int64_t hw = m->desc.hidden_width, nh = m->desc.hidden_layers;
    const struct { float** p; int64_t n; } a[] = {{&m->zbuf, B * m->H}, {&m->dz, B * 16}, {&m->acts, B * hw * nh},
                                                  {&m->delta, B * hw * nh}, {&m->enc, m->bwd_chunk * m->E}};
    for (auto& x : a)
        if (hipMalloc((void**)x.p, sizeof(float) * (size_t)std::max<int64_t>(x.n, 1)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(NIF_E_OOM, "training scratch allocation failed");
        }
    {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        int64_t need = 0;
        for (int i = 0; i < m->n_layers; ++i) {
            const bool out = i == m->n_layers - 1;
            need = std::max(need, dw_part_floats_max(out ? 16 : (int)hw, m->dims[i], cus));
        }
        if (m->dw_part) { (void)hipFree(m->dw_part); m->dw_part = nullptr; }
        for (void** p : {(void**)&m->ord_u32, (void**)&m->ord_f32, (void**)&m->ord_temp})
            if (*p) { (void)hipFree(*p); *p = nullptr; }
        m->ord_temp_bytes = order_temp_bytes(B);
        if (m->ord_temp_bytes == 0 ||
            hipMalloc((void**)&m->ord_u32, sizeof(uint32_t) * 4 * (size_t)B) != hipSuccess ||
            hipMalloc((void**)&m->ord_f32, sizeof(float) * 15 * (size_t)B) != hipSuccess ||
            hipMalloc(&m->ord_temp, m->ord_temp_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(NIF_E_OOM, "batch-ordering scratch allocation failed");
        }
        if (hipMalloc((void**)&m->dw_part, sizeof(float) * (size_t)need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(NIF_E_OOM, "weight-gradient scratch allocation failed");
        }
        m->dw_part_n = need;
    }
    m->max_batch = B;
    return NIF_OK;
}

int model_reserve_encoding(nif_model* m) {
    if (m->max_batch <= 0) return fail(NIF_E_STATE, "nif_model_reserve must come first");
    if (m->enc_all) return NIF_OK;
    if (hipMalloc((void**)&m->enc_all, sizeof(float) * (size_t)m->max_batch * m->E) != hipSuccess) {
        (void)hipGetLastError();
        m->enc_all = nullptr;
        return fail(NIF_E_OOM, "stored-encoding allocation failed");
    }
    return NIF_OK;
}

// ------------------------------------------------------------------ small kernels

__global__ void k_zero_f32(float* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = 0.f;
}

__global__ void k_train_begin(double* dacc, int64_t* tcount, float scale_init) {
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 5; ++k) dacc[DA_SUM + k] = 0.0;
    tcount[TC_NPOS] = 0;
    tcount[TC_NONFINITE] = 0;
    if (!(dacc[DA_SCALE] > 0.0)) dacc[DA_SCALE] = scale_init;
    dacc[DA_SCALE_USED] = dacc[DA_SCALE];
}

__global__ void k_count_pos(const uint8_t* __restrict__ hit, int64_t B, int64_t* tcount) {
    int64_t c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < B; i += (int64_t)gridDim.x * blockDim.x) c += hit[i] ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane_id() == 0 && c) atomicAdd((unsigned long long*)&tcount[TC_NPOS], (unsigned long long)c);
}

__global__ void k_pad_dz(const float* __restrict__ dh, int H, int64_t B, float* __restrict__ dz) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < B * 16; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / 16;
        const int h = (int)(i % 16);
        dz[i] = h < H ? dh[r * H + h] : 0.f;
    }
}

__device__ __forceinline__ float sigm(float v) { return 1.f / (1.f + expf(-v)); }

// Per-sample loss terms and d loss / d heads (times the loss scale), padded to 16 columns.
// Rows [0, n) of a batch of Btot samples (means over Btot and over its positives); label and
// point pointers start at the chunk, SoA arrays with stride ld.
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ z, int H, int64_t n, int64_t ld, int64_t Btot,
                                              const uint8_t* __restrict__ lhit, const float* __restrict__ lt,
                                              const float* __restrict__ ln, const float* __restrict__ la,
                                              const int32_t* __restrict__ lm, const float* __restrict__ s,
                                              const int64_t* __restrict__ tcount, double* __restrict__ dacc,
                                              float* __restrict__ dz, int dz_ld, const float* __restrict__ x0,
                                              const float* __restrict__ x1, int dist_head, int fixed) {
    const int M = H - 8;
    const double P = (double)tcount[TC_NPOS];
    const float scale = (float)dacc[DA_SCALE_USED];
    float w0 = expf(-s[0]), w1 = 0.5f * expf(-s[1]), w2 = 0.5f * expf(-s[2]), w3 = 0.5f * expf(-s[3]),
          w4 = expf(-s[4]);
    if (fixed) w0 = w1 = w2 = w3 = w4 = 1.f;
    const float invB = (float)(1.0 / (double)Btot), invP = P > 0 ? (float)(1.0 / P) : 0.f;
    const int64_t B = ld;                      // stride of the SoA label / point arrays
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float* zi = z + i * H;
        float g[16];
#pragma unroll
        for (int h = 0; h < 16; ++h) g[h] = 0.f;
        const float y = lhit[i] ? 1.f : 0.f;
        const float z0 = zi[0];
        acc[0] += fmaxf(z0, 0.f) - z0 * y + log1pf(expf(-fabsf(z0)));
        g[0] = w0 * (sigm(z0) - y) * invB;
        if (lhit[i] && P > 0) {
            if (dist_head == NIF_DIST_SIGMOID) {
                const float ex = x1[i] - x0[i], ey = x1[B + i] - x0[B + i], ez = x1[2 * B + i] - x0[2 * B + i];
                const float lr = sqrtf(ex * ex + ey * ey + ez * ez);
                const float tau = lr > 0.f ? fminf(fmaxf(lt[i] / lr, 0.f), 1.f) : 0.f;
                const float p = sigm(zi[1]);
                const float r = p - tau;
                acc[1] += (double)r * r;
                g[1] = w1 * 2.f * r * p * (1.f - p) * invP;
            } else {
                const float dh = fmaxf(zi[1], 0.f);
                const float r = logf(dh + kDistEps) - logf(lt[i] + kDistEps);
                acc[1] += (double)r * r;
                if (zi[1] > 0.f) g[1] = w1 * 2.f * r / (dh + kDistEps) * invP;
            }
            const float nt[3] = {ln[i], ln[B + i], ln[2 * B + i]};
            const float v[3] = {zi[2], zi[3], zi[4]};
            const float vl = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            const float den = fmaxf(vl, 1e-12f);
            const float nh[3] = {v[0] / den, v[1] / den, v[2] / den};
            const float c = nh[0] * nt[0] + nh[1] * nt[1] + nh[2] * nt[2];
            acc[2] += 1.0 - c;
#pragma unroll
            for (int a = 0; a < 3; ++a) g[2 + a] = w2 * (vl > 1e-12f ? -(nt[a] - nh[a] * c) / vl : -nt[a] / 1e-12f) * invP;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float ah = sigm(zi[5 + a]);
                const float df = ah - la[a * B + i];
                acc[3] += fabsf(df) / 3.0;
                const float sg = df > 0.f ? 1.f : (df < 0.f ? -1.f : 0.f);
                g[5 + a] = w3 * sg * ah * (1.f - ah) * invP / 3.f;
            }
            if (M == 1) {
                const float ym = lm[i] ? 1.f : 0.f;
                acc[4] += fmaxf(zi[8], 0.f) - zi[8] * ym + log1pf(expf(-fabsf(zi[8])));
                g[8] = w4 * (sigm(zi[8]) - ym) * invP;
            } else {
                const int mi = min(max(lm[i], 0), M - 1);   // ids outside [0, M) are clamped
                float mx = zi[8];
                for (int c2 = 1; c2 < M; ++c2) mx = fmaxf(mx, zi[8 + c2]);
                float se = 0.f;
                for (int c2 = 0; c2 < M; ++c2) se += expf(zi[8 + c2] - mx);
                const float lse = mx + logf(se);
                acc[4] += lse - zi[8 + mi];
#pragma unroll
                for (int c2 = 0; c2 < 8; ++c2)
                    if (c2 < M) g[8 + c2] = w4 * (expf(zi[8 + c2] - lse) - (c2 == mi ? 1.f : 0.f)) * invP;
            }
        }
        if (dz_ld == 16) {
            float4* dst = reinterpret_cast<float4*>(dz + i * 16);
#pragma unroll
            for (int h = 0; h < 4; ++h) dst[h] = make_float4(scale * g[4 * h], scale * g[4 * h + 1], scale * g[4 * h + 2], scale * g[4 * h + 3]);
        } else if (dz) {
#pragma unroll
            for (int h = 0; h < 16; ++h)
                if (h < H) dz[i * dz_ld + h] = scale * g[h];
        }
    }
    __shared__ double red[4][5];
#pragma unroll
    for (int k = 0; k < 5; ++k)
        for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0)
        for (int k = 0; k < 5; ++k) red[w][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < 5) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i][threadIdx.x];
        atomicAdd(&dacc[DA_SUM + threadIdx.x], t);
    }
}

// ------------------------------------------------------------------ MLP backward (MFMA)

struct BwdParams {
    const void* Wt[kMaxLayers];   // transposed padded weights of layers >= 1, [in][out_pad]
    int32_t n_hidden;
};

// delta[k][seg][HW] = d loss / d pre-activation of hidden layer k, chained from dz through the
// transposed weights: d in^T = W^T x d out^T, then masked by ReLU'(stored activation).
template <int HW, int PREC>
__global__ void __launch_bounds__(256) k_mlp_bwd(BwdParams bp, const float* __restrict__ dz,
                                                 const float* __restrict__ acts, float* __restrict__ delta,
                                                 int64_t B) {
    constexpr int CB = HW >= 128 ? 2 : 4;
    constexpr int OB = HW / 16;
    const int lane = lane_id(), q = lane >> 4, j = lane & 15;
    const int64_t per_tile = 16 * CB;
    const int64_t n_tiles = (B + per_tile - 1) / per_tile;
    const int64_t wave_g = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t tile = wave_g; tile < n_tiles; tile += n_waves) {
        const int64_t seg0 = tile * per_tile;
        floatx4 dh[OB][CB];
        // output layer: d out from dz (16 padded outputs)
        {
            floatx4 dout[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int64_t seg = seg0 + cb * 16 + j;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (seg < B) v = *reinterpret_cast<const float4*>(dz + seg * 16 + 4 * q);
                dout[cb] = floatx4{v.x, v.y, v.z, v.w};
            }
            shortx4 pout[CB];
            if constexpr (PREC != P_FP32) {
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) pout[cb] = pack4<PREC>(dout[cb][0], dout[cb][1], dout[cb][2], dout[cb][3]);
            }
#pragma unroll
            for (int ib = 0; ib < OB; ++ib)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                    if constexpr (PREC == P_FP32) {
                        const float4 wv = *reinterpret_cast<const float4*>(
                            reinterpret_cast<const float*>(bp.Wt[bp.n_hidden]) + (size_t)(ib * 16 + j) * 16 + 4 * q);
                        const float wf[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc = mfma32(wf[r], dout[cb][r], acc);
                    } else {
                        const shortx4 wa = *reinterpret_cast<const shortx4*>(
                            reinterpret_cast<const uint16_t*>(bp.Wt[bp.n_hidden]) + (size_t)(ib * 16 + j) * 16 + 4 * q);
                        acc = mfma16<PREC>(wa, pout[cb], acc);
                    }
                    dh[ib][cb] = acc;
                }
        }
        for (int k = bp.n_hidden - 1;; --k) {
            // mask with ReLU'(h_k) and store delta_k
#pragma unroll
            for (int ib = 0; ib < OB; ++ib)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int64_t seg = seg0 + cb * 16 + j;
                    if (seg < B) {
                        const size_t o = ((size_t)k * B + seg) * HW + ib * 16 + 4 * q;
                        const float4 a = *reinterpret_cast<const float4*>(acts + o);
                        dh[ib][cb][0] = a.x > 0.f ? dh[ib][cb][0] : 0.f;
                        dh[ib][cb][1] = a.y > 0.f ? dh[ib][cb][1] : 0.f;
                        dh[ib][cb][2] = a.z > 0.f ? dh[ib][cb][2] : 0.f;
                        dh[ib][cb][3] = a.w > 0.f ? dh[ib][cb][3] : 0.f;
                        *reinterpret_cast<float4*>(delta + o) = make_float4(dh[ib][cb][0], dh[ib][cb][1], dh[ib][cb][2], dh[ib][cb][3]);
                    } else {
                        dh[ib][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
                    }
                }
            if (k == 0) break;
            // through hidden layer k (affine layer k: hidden k-1 -> hidden k)
            floatx4 dn[OB][CB];
#pragma unroll
            for (int ib = 0; ib < OB; ++ib)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) dn[ib][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
            // the deltas as B operands, converted once for all output blocks
            shortx4 pk[OB][CB];
            if constexpr (PREC != P_FP32) {
#pragma unroll
                for (int ob = 0; ob < OB; ++ob)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        pk[ob][cb] = pack4<PREC>(dh[ob][cb][0], dh[ob][cb][1], dh[ob][cb][2], dh[ob][cb][3]);
            }
#pragma unroll
            for (int ib = 0; ib < OB; ++ib)
#pragma unroll
                for (int ob = 0; ob < OB; ++ob) {
                    if constexpr (PREC == P_FP32) {
                        const float4 wv = *reinterpret_cast<const float4*>(
                            reinterpret_cast<const float*>(bp.Wt[k]) + (size_t)(ib * 16 + j) * HW + ob * 16 + 4 * q);
                        const float wf[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb) dn[ib][cb] = mfma32(wf[r], dh[ob][cb][r], dn[ib][cb]);
                    } else {
                        const shortx4 wa = *reinterpret_cast<const shortx4*>(
                            reinterpret_cast<const uint16_t*>(bp.Wt[k]) + (size_t)(ib * 16 + j) * HW + ob * 16 + 4 * q);
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) dn[ib][cb] = mfma16<PREC>(wa, pk[ob][cb], dn[ib][cb]);
                    }
                }
#pragma unroll
            for (int ib = 0; ib < OB; ++ib)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) dh[ib][cb] = dn[ib][cb];
        }
    }
}


// Weight gradient dW = D^T H of one layer as K-sliced partial sums on MFMA, read straight
// from the row-major [K][*] operands.  A wave owns MT 16-row tiles x 4 16-column tiles
// (MT = M_pad / 16) with a permuted mapping that makes every operand fetch contiguous: MFMA
// row r of tile mt is output row MT r + mt and column c of tile nt is output column
// n0 + 4c + nt, so lane (q, j) reads D[k][MT j .. MT j + MT) and H[k][n0 + 4j .. + 4) of its
// own k (one k per lane quarter q).  Block (x, y): K chunk x, column group y of 4 x 64
// columns; when the layer has fewer than 4 column tiles, the spare waves take further
// slices of the chunk.  Partials (and the bias sums of column group 0) go to a scratch slot
// per (chunk, slice); k_dw_sum adds the slots into the gradient, without atomics.
template <int MT, int PREC>
__global__ void __launch_bounds__(256) k_dw_part(DwArgs A) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, j = lane & 15;
    const int cb = A.ks > 1 ? w % A.n_cb : (int)blockIdx.y * 4 + w;      // column tile
    const int sub = A.ks > 1 ? w / A.n_cb : 0;                           // K slice within the chunk
    if (cb >= A.n_cb || sub >= A.ks) return;
    const int64_t kc0 = (int64_t)blockIdx.x * A.Kc, kc1 = std::min<int64_t>(A.B, kc0 + A.Kc);
    const int64_t ksz = (A.Kc + A.ks - 1) / A.ks;
    const int64_t k0 = kc0 + sub * ksz, k1 = std::min<int64_t>(kc1, k0 + ksz);
    const int n0 = cb * 64;
    floatx4 acc[MT][4];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bs[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) bs[a] = 0.f;
    const bool ncol_ok = n0 + 4 * j + 3 < A.N;
    // FP32: one 16x16x4 MFMA per 4 samples, lane quarter q holding sample q of each group.
    // BF16/FP16: operands rounded from the stored FP32 deltas and activations, one 16x16x16
    // MFMA per 16 samples, lane quarter q holding samples 4q .. 4q + 3 (same row and column
    // mapping).
    constexpr int R = PREC == P_FP32 ? 1 : 4;
    constexpr int STEP = 4 * R;
    float av[R][MT], bv[R][4];
    auto load = [&](int64_t kb, float (&a)[R][MT], float (&b)[R][4]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t k = kb + R * q + r;
            if (k < k1) {
                const float* dr = A.d + k * A.dstride + MT * j;
                if constexpr (MT >= 4) {
#pragma unroll
                    for (int t = 0; t < MT; t += 4) {
                        const float4 v = *reinterpret_cast<const float4*>(dr + t);
                        a[r][t] = v.x; a[r][t + 1] = v.y; a[r][t + 2] = v.z; a[r][t + 3] = v.w;
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < MT; ++t) a[r][t] = dr[t];
                }
                const float* hr = A.h + k * A.hstride + n0 + 4 * j;
                if (ncol_ok) {
                    const float4 v = *reinterpret_cast<const float4*>(hr);
                    b[r][0] = v.x; b[r][1] = v.y; b[r][2] = v.z; b[r][3] = v.w;
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) b[r][t] = n0 + 4 * j + t < A.N ? hr[t] : 0.f;
                }
            } else {
#pragma unroll
                for (int t = 0; t < MT; ++t) a[r][t] = 0.f;
#pragma unroll
                for (int t = 0; t < 4; ++t) b[r][t] = 0.f;
            }
        }
    };
    for (int64_t kb = k0; kb < k1; kb += STEP) {
        load(kb, av, bv);
        if constexpr (PREC == P_FP32) {
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                bs[a] += av[0][a];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] = mfma32(av[0][a], bv[0][c], acc[a][c]);
            }
        } else {
            shortx4 bp[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) bp[c] = pack4<PREC>(bv[0][c], bv[1][c], bv[2][c], bv[3][c]);
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                bs[a] += (av[0][a] + av[1][a]) + (av[2][a] + av[3][a]);
                const shortx4 ap = pack4<PREC>(av[0][a], av[1][a], av[2][a], av[3][a]);
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] = mfma16<PREC>(ap, bp[c], acc[a][c]);
            }
        }
    }
    const int64_t slot = (int64_t)blockIdx.x * A.ks + sub;
    float* P = A.part + slot * A.M_pad * A.N;
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = MT * (4 * q + r) + a;
            const int col = n0 + 4 * j;
            float* dst = P + (int64_t)row * A.N + col;
            if (ncol_ok) {
                *reinterpret_cast<float4*>(dst) = make_float4(acc[a][0][r], acc[a][1][r], acc[a][2][r], acc[a][3][r]);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (col + c < A.N) dst[c] = acc[a][c][r];
            }
        }
    if (cb == 0) {             // bias: sum of D over the slice, rows MT j + a (lanes of one j sum their k)
        float* pb = A.part + A.n_slots * A.M_pad * A.N + slot * A.M_pad;
#pragma unroll
        for (int a = 0; a < MT; ++a) {
            float v = bs[a];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (q == 0) pb[MT * j + a] = v;
        }
    }
}

// Weight gradient dW = D^T H of a layer with 64 RW output rows, staged through LDS.  Block
// (x, y) covers K chunk x and CT 64-column tiles starting at column 64 CT y, with RW x CT waves:
// wave (rw, ct) owns rows [64 rw, + 64) and columns [64 (CT y + ct), + 64) as 4 x 4 MFMA tiles
// (tile (a, c): rows 16a + 4q + r, columns 16c + j of the wave's).  The block's threads load
// each 16-sample tile of D [16][64 RW] and H [16][64 CT] with coalesced float4 loads into
// registers while the waves multiply the previous tile out of LDS (double buffer, one barrier
// per tile), so a tile's loads are in flight behind a whole tile of MFMAs and each operand
// row is fetched once per block.  LDS rows are padded by 4 floats, so the column reads of the
// four lane quarters (4 rows apart) fall in distinct banks.  Partials (and the bias sums, by
// the waves of column tile 0) go to slot x; k_dw_sum adds the slots.  Needs N % 4 == 0.
template <int RW, int CT, int PREC>
__global__ void __launch_bounds__(64 * RW * CT) __attribute__((amdgpu_waves_per_eu(3))) k_dw_tile(DwArgs A) {
    constexpr int NT = 64 * RW * CT;
    constexpr int M = 64 * RW, LDD = M + 4;
    constexpr int NC = 64 * CT, LDH = NC + 4;
    constexpr int F4D = kDwKT * M / 4, F4H = kDwKT * NC / 4;
    constexpr int NLD = (F4D + F4H + NT - 1) / NT;
    __shared__ float sD[2][kDwKT * LDD];
    __shared__ float sH[2][kDwKT * LDH];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, q = lane >> 4, j = lane & 15;
    const int rw = w / CT, ct = w % CT;
    const int64_t kc0 = (int64_t)blockIdx.x * A.Kc, kc1 = std::min<int64_t>(A.B, kc0 + A.Kc);
    const int col0 = (int)blockIdx.y * NC;
    const int cb = (int)blockIdx.y * CT + ct;
    const bool live = cb < A.n_cb;
    const int n_tiles = (int)((kc1 - kc0 + kDwKT - 1) / kDwKT);
    float4 reg[NLD];
    auto load = [&](int t) {
        const int64_t kt = kc0 + (int64_t)t * kDwKT;
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int idx = tid + i * NT;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (idx < F4D) {
                const int r = idx / (M / 4), c4 = idx % (M / 4);
                const int64_t k = kt + r;
                if (k < kc1) v = *reinterpret_cast<const float4*>(A.d + k * A.dstride + 4 * c4);
            } else if (idx < F4D + F4H) {
                const int h = idx - F4D, r = h / (NC / 4), c4 = h % (NC / 4);
                const int64_t k = kt + r;
                const int col = col0 + 4 * c4;
                if (k < kc1 && col < A.N) v = *reinterpret_cast<const float4*>(A.h + k * A.hstride + col);
            }
            reg[i] = v;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int idx = tid + i * NT;
            if (idx < F4D) {
                const int r = idx / (M / 4), c4 = idx % (M / 4);
                *reinterpret_cast<float4*>(&sD[buf][r * LDD + 4 * c4]) = reg[i];
            } else if (idx < F4D + F4H) {
                const int h = idx - F4D, r = h / (NC / 4), c4 = h % (NC / 4);
                *reinterpret_cast<float4*>(&sH[buf][r * LDH + 4 * c4]) = reg[i];
            }
        }
    };
    floatx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bs[4] = {0.f, 0.f, 0.f, 0.f};
    const int dc = 64 * rw + j;                // this lane's row within the block's D tile
    const int hc = 64 * ct + j;                // this lane's column within the block's H tile
    if (n_tiles > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
#pragma unroll 1
    for (int t = 0; t < n_tiles; ++t) {
        const int cur = t & 1;
        if (t + 1 < n_tiles) load(t + 1);
        if (live) {
            const float* D = sD[cur];
            const float* H = sH[cur];
            if constexpr (PREC == P_FP32) {
#pragma unroll
                for (int st4 = 0; st4 < kDwKT / 4; ++st4) {
                    const int k = 4 * st4 + q;
                    float bv[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) bv[c] = H[k * LDH + hc + 16 * c];
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const float av = D[k * LDD + dc + 16 * a];
                        bs[a] += av;
#pragma unroll
                        for (int c = 0; c < 4; ++c) acc[a][c] = mfma32(av, bv[c], acc[a][c]);
                    }
                }
            } else {
                static_assert(kDwKT == 16, "one 16x16x16 MFMA step per tile");
                shortx4 bp[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float* hp = H + 4 * q * LDH + hc + 16 * c;
                    bp[c] = pack4<PREC>(hp[0], hp[LDH], hp[2 * LDH], hp[3 * LDH]);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const float* dp = D + 4 * q * LDD + dc + 16 * a;
                    const float d0 = dp[0], d1 = dp[LDD], d2 = dp[2 * LDD], d3 = dp[3 * LDD];
                    bs[a] += (d0 + d1) + (d2 + d3);
                    const shortx4 ap = pack4<PREC>(d0, d1, d2, d3);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[a][c] = mfma16<PREC>(ap, bp[c], acc[a][c]);
                }
            }
        }
        if (t + 1 < n_tiles) store(cur ^ 1);
        __syncthreads();
    }
    if (!live) return;
    const int64_t slot = blockIdx.x;
    float* P = A.part + slot * A.M_pad * A.N;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 64 * rw + 16 * a + 4 * q + r;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int col = 64 * cb + 16 * c + j;
                if (col < A.N) P[(int64_t)row * A.N + col] = acc[a][c][r];
            }
        }
    if (cb == 0) {             // bias: sum of D over the chunk, row 64 rw + 16a + j (lanes of one j sum their k)
        float* pb = A.part + A.n_slots * A.M_pad * A.N + slot * A.M_pad;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            float v = bs[a];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (q == 0) pb[64 * rw + 16 * a + j] = v;
        }
    }
}

// gW[m][n] += sum over slots of part[slot][m][n] (m < M_real), gb[m] likewise.  Block: 64
// consecutive outputs x kDwSumGroups groups of slots (the groups' sums meet in LDS), so each
// thread's chain of dependent loads is n_slots / kDwSumGroups long.
constexpr int kDwSumGroups = 16;
__global__ void __launch_bounds__(64 * kDwSumGroups) k_dw_sum(DwArgs A, float* __restrict__ gW, int ldw, float* __restrict__ gb) {
    __shared__ float red[kDwSumGroups][64];
    const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t n_out = (int64_t)A.M_real * A.N;
    const int64_t i = (int64_t)blockIdx.x * 64 + o;
    const bool is_w = i < n_out, live = i < n_out + A.M_real;
    const float* p = nullptr;
    int64_t stride = 0;
    if (is_w) {
        p = A.part + (i / A.N) * A.N + i % A.N;
        stride = (int64_t)A.M_pad * A.N;
    } else if (live) {
        p = A.part + A.n_slots * A.M_pad * A.N + (i - n_out);
        stride = A.M_pad;
    }
    constexpr int G = kDwSumGroups;
    float s = 0.f;
    if (live) {
        int64_t t = g;
        float s1 = 0.f, s2 = 0.f, s3 = 0.f;
        for (; t + 3 * G < A.n_slots; t += 4 * G) {
            s += p[t * stride];
            s1 += p[(t + G) * stride];
            s2 += p[(t + 2 * G) * stride];
            s3 += p[(t + 3 * G) * stride];
        }
        for (; t < A.n_slots; t += G) s += p[t * stride];
        s += s1 + s2 + s3;
    }
    red[g][o] = s;
    __syncthreads();
    if (g == 0 && live) {
        float v = 0.f;
#pragma unroll
        for (int k = 0; k < G; ++k) v += red[k][o];
        if (is_w) gW[(i / A.N) * ldw + i % A.N] += v;
        else gb[i - n_out] += v;
    }
}


// ------------------------------------------------------------------ encoding backward
// The table gradient is a scatter-add: every (sample, PE combination, level, corner) adds
// w_corner * d enc to one table entry, about 2e9 additions per 2^18-sample step.  Device-
// scope float atomics on this part are executed past the per-XCD L2s and would bound the
// step, so the additions are grouped instead:
//   count  - each block histograms the table slices ("buckets", at most 4096 entries of one
//            level each) its additions fall into (LDS atomics) and stores the counts;
//   scan   - an exclusive scan over (bucket, block) gives every block a private output range
//            per bucket;
//   fill   - the same block decomposition recomputes the additions and writes (entry within
//            the slice, value pair) into its ranges (LDS cursors, no global atomics);
//   reduce - one block per part of a slice sums its additions in LDS and adds them to the
//            FP32 table gradient.
// Lanes are assigned as in the forward's first layer: lane (q, j) takes sample j of a
// 16-sample tile and PE combination c = 4u + q; the wave walks the levels in pairs, all
// lanes on the same level.  d enc = W0^T delta_0 is formed on MFMA in the same layout: the
// 16 output rows of one step are (combination 4u + r/4, features of the level pair), so
// lane (q, j) receives exactly the four d enc values of its own combination and sample.
// dW0 comes from the stored encoding (k_dw_part, k_dw_sum).  Samples are processed in chunks so the
// addition buffer stays bounded.

struct EncBwdParams {
    EncParams enc;
    const float* W0t;    // FP32 [E][HW]: W0 transposed
    const float* delta0; // [rows][HW]; row of sample seg = seg - drow0
    int64_t drow0;
    const float* x0;     // SoA [3][B]
    const float* x1;
    int32_t HW, E, S;
    float* g_tables;
    float* dx0;          // nullable SoA [3][B]
    float* dx1;
    int64_t B;           // stride of the SoA point arrays
    int64_t c0;          // first sample of this round
    int64_t n;           // samples in this round
    int32_t SB;          // log2 entries per bucket
    int32_t NBL;         // buckets per level
    int32_t n_buckets;   // L * NBL
    int32_t n_blk;       // blocks of the round's grid
    int32_t blk0;        // fill: the launch's first block within the round
    int32_t* cnt;        // [n_buckets][n_blk] counts, then exclusive offsets
    float* val;          // table-gradient records, kRecFloats floats each (see below)
    int32_t w_lds;       // fill: the block's first-layer weight rows staged in LDS
    int64_t cap;         // capacity of val, in records
    uint32_t* vmax;      // bits of a bound on the round's |additions| (+inf if one is not finite)
};


// Table-gradient records, 16 bytes each.  Three features: one addition (v0, v1, v2, entry
// within the bucket as bits).  Two features: the additions of an x-neighbour corner pair, whose
// trilinear weights share the y and z factors A: (a0, a1) = A d enc, w = the x weight of the
// upper corner, and both entries k0 | k1 << 16; the lower corner receives (1 - w) a, the upper
// w a.  A pair whose corners fall into different buckets is written as two records with k0 = k1,
// w = 0 and a pre-multiplied by the corner's x factor.
__device__ __forceinline__ uint32_t pair_key(uint32_t k0, uint32_t k1) { return k0 | (k1 << 16); }

// Sample position, d position / d x and the in-range mask of PE combination c (point-major).
__device__ __forceinline__ void pe_combo_grad(const float xs[6], int c, int S, double smp[3], float dsdx[3],
                                              float inside[3]) {
    const int p = c >= S ? 1 : 0;
    const int s = c - p * S;
    const int k = s > 0 ? (s - 1) >> 1 : 0;
    const double f = ldexp(1.0, k);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float xv = xs[3 * p + a];
        inside[a] = (xv >= 0.f && xv <= 1.f) ? 1.f : 0.f;
        const double v = fmin(fmax((double)xv, 0.0), 1.0);
        double sn, cs;
        sincos(f * v, &sn, &cs);
        if (s == 0) { smp[a] = v; dsdx[a] = 1.f; }
        else if (s & 1) { smp[a] = 0.5 * (sn + 1.0); dsdx[a] = (float)(0.5 * f * cs); }
        else { smp[a] = 0.5 * (cs + 1.0); dsdx[a] = (float)(-0.5 * f * sn); }
    }
}

// The 8 corner entries (within the level) and trilinear weights of one level at smp.
__device__ __forceinline__ void level_corners(const EncParams& ep, int l, const double smp[3], uint32_t idx[8],
                                              float wx[3]) {
    const int N = ep.res[l];
    const uint32_t mask = (1u << ep.log2T) - 1u;
    uint32_t ix, iy, iz;
    grid_axis(smp[0], N, ix, wx[0]);
    grid_axis(smp[1], N, iy, wx[1]);
    grid_axis(smp[2], N, iz, wx[2]);
    const bool dense = (ep.dense_mask >> l) & 1u;
    const uint32_t n1 = (uint32_t)N + 1u;
#pragma unroll
    for (int cc = 0; cc < 8; ++cc)
        idx[cc] = grid_index(ix + (cc & 1), iy + ((cc >> 1) & 1), iz + ((cc >> 2) & 1), n1, dense, mask);
}

__device__ __forceinline__ float corner_weight(const float w[3], int cc) {
    return ((cc & 1) ? w[0] : 1.f - w[0]) * (((cc >> 1) & 1) ? w[1] : 1.f - w[1]) * (((cc >> 2) & 1) ? w[2] : 1.f - w[2]);
}

// Sample of lane j in tile `tile` of the chunk, its points (x0 then x1) and validity.
__device__ __forceinline__ bool tile_sample(const EncBwdParams& P, int64_t tile, int j, int64_t& seg, float xs[6]) {
    seg = P.c0 + tile * 16 + j;
    const bool valid = tile * 16 + j < P.n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        xs[a] = valid ? P.x0[a * P.B + seg] : 0.5f;
        xs[3 + a] = valid ? P.x1[a * P.B + seg] : 0.5f;
    }
    return valid;
}

// Largest dynamic LDS of a fill block that stages its first-layer rows (else they are read from
// memory for every tile).
constexpr size_t kFillLdsMax = 60 * 1024;

// Levels per block row of the count and fill passes: two with two features per entry (the
// four (level, feature) rows of a PE combination), one with three.
template <int FD> constexpr int kLevelGroup = FD == 2 ? 2 : 1;

// Buckets of one level group: table set s (one per PE sample with per-sample tables, else one),
// level lp + k, slice: local index (s LG + k) NBL + slice, global ((s L + lp + k) NBL + slice).
template <int LG>
__device__ __forceinline__ int64_t group_bucket_global(const EncBwdParams& P, int lp, int i) {
    const int s = i / (LG * P.NBL), r = i % (LG * P.NBL);
    return ((int64_t)s * P.enc.L + lp + r / P.NBL) * P.NBL + r % P.NBL;
}
__device__ __forceinline__ int n_table_sets(const EncBwdParams& P) { return P.enc.set_stride ? P.S : 1; }
// Table set of PE combination c (point-major).
__device__ __forceinline__ int combo_set(const EncBwdParams& P, int c) {
    return P.enc.set_stride ? (c >= P.S ? c - P.S : c) : 0;
}

// Block (x, y): the samples of tile group x, the levels of level group y (as the fill below).
template <int FD>
__global__ void __launch_bounds__(256) k_enc_bwd_count(EncBwdParams P) {
    constexpr int LG = kLevelGroup<FD>;
    extern __shared__ int32_t s_h[];    // [sets][LG][NBL]
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, q = lane >> 4, j = lane & 15;
    const int n_comb = 2 * P.S;
    const int lp = (int)blockIdx.y * LG;
    const int nloc = LG * P.NBL * n_table_sets(P);
    for (int i = tid; i < nloc; i += 256) s_h[i] = 0;
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) *P.vmax = 0u;
    __syncthreads();
    const int64_t n_tiles = (P.n + 15) / 16;
    const int64_t t_end = std::min<int64_t>(n_tiles, (int64_t)(blockIdx.x + 1) * kBwdTilesPerBlock);
    for (int64_t tile = (int64_t)blockIdx.x * kBwdTilesPerBlock + w; tile < t_end; tile += 4) {
        int64_t seg;
        float xs[6];
        const bool valid = tile_sample(P, tile, j, seg, xs);
        for (int u = 0; 4 * u < n_comb; ++u) {
            const int c = 4 * u + q;
            const bool live = valid && c < n_comb;
            double smp[3];
            float dsdx[3], inside[3];
            pe_combo_grad(xs, live ? c : 0, P.S, smp, dsdx, inside);
            const int sb = combo_set(P, live ? c : 0) * LG;
            for (int k = 0; k < LG; ++k) {
                uint32_t idx[8];
                float wt[3];
                level_corners(P.enc, lp + k, smp, idx, wt);
                if (!live) continue;
                int32_t* h = s_h + (sb + k) * P.NBL;
                if constexpr (FD == 2) {
#pragma unroll
                    for (int pr = 0; pr < 4; ++pr) {
                        const int b0 = (int)(idx[2 * pr] >> P.SB), b1 = (int)(idx[2 * pr + 1] >> P.SB);
                        atomicAdd(&h[b0], 1);
                        if (b1 != b0) atomicAdd(&h[b1], 1);
                    }
                } else {
#pragma unroll
                    for (int cc = 0; cc < 8; ++cc) atomicAdd(&h[(int)(idx[cc] >> P.SB)], 1);
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < nloc; i += 256) P.cnt[group_bucket_global<LG>(P, lp, i) * P.n_blk + blockIdx.x] = s_h[i];
}

// Block (x, y): the samples of tile group x, the LG levels of level group y only, so that a
// block writes into the LG NBL buckets of those levels: the lines it leaves partly written at
// any time stay few enough to complete in L2 before eviction.
template <int HW, int FD>
__global__ void __launch_bounds__(256) k_enc_bwd_fill(EncBwdParams P) {
    constexpr int KQ = HW / 4;                 // MFMA k-steps: lane quarter q covers [q KQ, (q+1) KQ)
    constexpr int LG = kLevelGroup<FD>;
    extern __shared__ int32_t s_cur[];         // [sets][LG][NBL]: this block's next output slot per bucket
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, q = lane >> 4, j = lane & 15;
    const int L = P.enc.L, n_comb = 2 * P.S;
    const int lp = (int)blockIdx.y * LG;       // first level of this block's group
    const uint32_t kmask = (1u << P.SB) - 1u;
    const int nloc = LG * P.NBL * n_table_sets(P);
    const int bx = (int)blockIdx.x + P.blk0;   // block within the round
    for (int i = tid; i < nloc; i += 256) s_cur[i] = P.cnt[group_bucket_global<LG>(P, lp, i) * P.n_blk + bx];
    // The W0 rows this block multiplies (combination c, (level, feature) r of its group: row
    // 4c + r, zero where r >= LG FD), staged once in LDS with rows padded by 4 floats, so the
    // MFMA's A operand is read from LDS rather than fetched again for every tile.
    constexpr int LDW = HW + 4;
    float* s_w = reinterpret_cast<float*>(s_cur + ((nloc + 3) & ~3));
    if (P.w_lds) {
        for (int i = tid; i < 4 * n_comb * (HW / 4); i += 256) {
            const int r = i / (HW / 4), c4 = i % (HW / 4);
            const int ca = r >> 2, fr = r & 3;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (fr < LG * FD) v = *reinterpret_cast<const float4*>(P.W0t + ((size_t)(ca * L + lp) * FD + fr) * HW + 4 * c4);
            *reinterpret_cast<float4*>(s_w + r * LDW + 4 * c4) = v;
        }
    }
    __syncthreads();
    const int64_t n_tiles = (P.n + 15) / 16;
    const int64_t t_end = std::min<int64_t>(n_tiles, (int64_t)(bx + 1) * kBwdTilesPerBlock);
    for (int64_t tile = (int64_t)bx * kBwdTilesPerBlock + w; tile < t_end; tile += 4) {
        int64_t seg;
        float xs[6];
        const bool valid = tile_sample(P, tile, j, seg, xs);
        // B operand: delta_0 of sample j, entries [q KQ, (q+1) KQ)
        float bd[KQ];
#pragma unroll
        for (int t = 0; t < KQ; t += 4) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (valid) v = *reinterpret_cast<const float4*>(P.delta0 + (seg - P.drow0) * HW + q * KQ + t);
            bd[t] = v.x; bd[t + 1] = v.y; bd[t + 2] = v.z; bd[t + 3] = v.w;
        }
        float dxa[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
        float vmx = 0.f;                       // largest |addition| of this lane (inf if not finite)
        for (int u = 0; 4 * u < n_comb; ++u) {
            const int c = 4 * u + q;
            const bool live = valid && c < n_comb;
            double smp[3];
            float dsdx[3], inside[3];
            pe_combo_grad(xs, live ? c : 0, P.S, smp, dsdx, inside);
            float dpos[3] = {0.f, 0.f, 0.f};
            // A operand row of lane (q, j): combination 4u + j/4, (level, feature) j%4 of the level
            // group in encoding order (with three features, index 3 is a zero row)
            const int ca = 4 * u + (j >> 2);
            const bool a_live = ca < n_comb && (j & 3) < LG * FD;
            {
                const int l0 = lp;
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                const float* wrow = P.w_lds ? s_w + (size_t)(a_live ? 4 * ca + (j & 3) : 0) * LDW + q * KQ
                                            : P.W0t + (size_t)(a_live ? (ca * L + l0) * FD + (j & 3) : 0) * HW + q * KQ;
#pragma unroll
                for (int t = 0; t < KQ; t += 4) {
                    float4 av = *reinterpret_cast<const float4*>(wrow + t);
                    if (!a_live) av = make_float4(0.f, 0.f, 0.f, 0.f);
                    acc = mfma32(av.x, bd[t], acc);
                    acc = mfma32(av.y, bd[t + 1], acc);
                    acc = mfma32(av.z, bd[t + 2], acc);
                    acc = mfma32(av.w, bd[t + 3], acc);
                }
                // acc[FD k + f] = d enc of (combination c, level l0 + k, feature f), sample j
#pragma unroll
                for (int k = 0; k < LG; ++k) {
                    const int l = l0 + k;
                    uint32_t idx[8];
                    float wt[3];
                    level_corners(P.enc, l, smp, idx, wt);
                    if (!live) continue;
                    float gf[FD];
#pragma unroll
                    for (int f = 0; f < FD; ++f) gf[f] = acc[FD * k + f];
                    float dl[3] = {0.f, 0.f, 0.f};
                    int32_t* cur = s_cur + (combo_set(P, c) * LG + l - lp) * P.NBL;
                    float amax = 0.f;
                    bool fin = true;
                    if constexpr (FD == 2) {
#pragma unroll
                        for (int pr = 0; pr < 4; ++pr) {
                            const int cl = 2 * pr;                 // lower-x corner; cl + 1 the upper
                            const float A = (((cl >> 1) & 1) ? wt[1] : 1.f - wt[1]) * (((cl >> 2) & 1) ? wt[2] : 1.f - wt[2]);
                            const float a0 = A * gf[0], a1 = A * gf[1];
                            const uint32_t k0 = idx[cl] & kmask, k1 = idx[cl + 1] & kmask;
                            const int b0 = (int)(idx[cl] >> P.SB), b1 = (int)(idx[cl + 1] >> P.SB);
                            fin = fin && isfinite(a0) && isfinite(a1);
                            amax = fmaxf(amax, fmaxf(fabsf(a0), fabsf(a1)));
                            if (b0 == b1) {
                                const int32_t slot = atomicAdd(&cur[b0], 1);
                                if (slot < P.cap)      // always true: the count pass saw the same records
                                    *reinterpret_cast<float4*>(P.val + (size_t)slot * kRecFloats) =
                                        make_float4(a0, a1, wt[0], __uint_as_float(pair_key(k0, k1)));
                            } else {
                                const float w0 = 1.f - wt[0];
                                const int32_t s0 = atomicAdd(&cur[b0], 1), s1 = atomicAdd(&cur[b1], 1);
                                if (s0 < P.cap)
                                    *reinterpret_cast<float4*>(P.val + (size_t)s0 * kRecFloats) =
                                        make_float4(w0 * a0, w0 * a1, 0.f, __uint_as_float(pair_key(k0, k0)));
                                if (s1 < P.cap)
                                    *reinterpret_cast<float4*>(P.val + (size_t)s1 * kRecFloats) =
                                        make_float4(wt[0] * a0, wt[0] * a1, 0.f, __uint_as_float(pair_key(k1, k1)));
                            }
                        }
                    } else {
#pragma unroll
                        for (int cc = 0; cc < 8; ++cc) {
                            const float cw = corner_weight(wt, cc);
                            const int32_t slot = atomicAdd(&cur[(int)(idx[cc] >> P.SB)], 1);
                            float v[FD];
#pragma unroll
                            for (int f = 0; f < FD; ++f) {
                                v[f] = cw * gf[f];
                                fin = fin && isfinite(v[f]);
                                amax = fmaxf(amax, fabsf(v[f]));
                            }
                            if (slot < P.cap)
                                *reinterpret_cast<float4*>(P.val + (size_t)slot * kRecFloats) =
                                    make_float4(v[0], v[1], v[2], __uint_as_float(idx[cc] & kmask));
                        }
                    }
                    vmx = fin ? fmaxf(vmx, amax) : INFINITY;
                    if (P.dx0) {
#pragma unroll
                        for (int cc = 0; cc < 8; ++cc) {
                            const size_t te = ((size_t)combo_set(P, c) * (size_t)P.enc.set_stride +
                                               ((size_t)l << P.enc.log2T) + idx[cc]) * FD;
                            float gd = 0.f;
#pragma unroll
                            for (int f = 0; f < FD; ++f) {
                                const float tv = P.enc.f16 ? __half2float(reinterpret_cast<const __half*>(P.enc.tab)[te + f])
                                                           : reinterpret_cast<const float*>(P.enc.tab)[te + f];
                                gd = fmaf(gf[f], tv, gd);
                            }
                            const float fx = (cc & 1) ? wt[0] : 1.f - wt[0];
                            const float fy = ((cc >> 1) & 1) ? wt[1] : 1.f - wt[1];
                            const float fz = ((cc >> 2) & 1) ? wt[2] : 1.f - wt[2];
                            dl[0] += gd * ((cc & 1) ? 1.f : -1.f) * fy * fz;
                            dl[1] += gd * (((cc >> 1) & 1) ? 1.f : -1.f) * fx * fz;
                            dl[2] += gd * (((cc >> 2) & 1) ? 1.f : -1.f) * fx * fy;
                        }
                    }
                    if (P.dx0) {
                        const float N = (float)P.enc.res[l];
#pragma unroll
                        for (int a = 0; a < 3; ++a) dpos[a] += dl[a] * N;
                    }
                }
            }
            if (P.dx0 && live) {
                const int p = c >= P.S ? 1 : 0;
#pragma unroll
                for (int a = 0; a < 3; ++a) dxa[p][a] += dpos[a] * dsdx[a] * inside[a];
            }
        }
        if (P.dx0 && valid)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                unsafeAtomicAdd(&P.dx0[a * P.B + seg], dxa[0][a]);
                unsafeAtomicAdd(&P.dx1[a * P.B + seg], dxa[1][a]);
            }
        for (int off = 32; off > 0; off >>= 1) vmx = fmaxf(vmx, __shfl_xor(vmx, off));
        if (lane == 0 && vmx > 0.f) atomicMax(P.vmax, __float_as_uint(vmx));   // non-negative: bits order as values
    }
}

// Exclusive scan of n int32 in place, in chunks of 4096: per-chunk sums, a one-block scan of
// the sums (total to *total), then per-chunk scans.
__global__ void __launch_bounds__(256) k_scan_sums(const int32_t* __restrict__ a, int64_t n, int32_t* __restrict__ sums) {
    __shared__ int32_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * 4096;
    int32_t acc = 0;
    for (int i = threadIdx.x; i < 4096; i += 256)
        if (base + i < n) acc += a[base + i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(1024) k_scan_top(int32_t* __restrict__ sums, int n_chunks, int32_t* __restrict__ total) {
    __shared__ int32_t sh[1024];
    int32_t carry = 0;
    for (int base = 0; base < n_chunks; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int32_t v = i < n_chunks ? sums[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int32_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n_chunks) sums[i] = carry + sh[threadIdx.x] - v;
        carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(256) k_scan_apply(int32_t* __restrict__ a, int64_t n, const int32_t* __restrict__ sums) {
    __shared__ int32_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * 4096 + (int64_t)threadIdx.x * 16;
    int32_t v[16];
    int32_t acc = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        v[k] = base + k < n ? a[base + k] : 0;
        acc += v[k];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int32_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = sums[blockIdx.x] + sh[threadIdx.x] - acc;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (base + k < n) a[base + k] = run;
        run += v[k];
    }
}

// Work list of the reduction: bucket b is cut into parts of at most kReducePart additions;
// parts[b] = exclusive prefix of the part counts (parts[n_buckets] = total parts).
constexpr int64_t kReducePart = 1 << 17;

__global__ void __launch_bounds__(1024) k_enc_bwd_parts(EncBwdParams P, const int32_t* __restrict__ total,
                                                        int32_t* __restrict__ parts) {
    __shared__ int32_t sh[1024];
    int32_t carry = 0;
    for (int base = 0; base < P.n_buckets; base += 1024) {
        const int b = base + (int)threadIdx.x;
        int32_t v = 0;
        if (b < P.n_buckets) {
            const int64_t start = P.cnt[(int64_t)b * P.n_blk];
            const int64_t end = b + 1 < P.n_buckets ? (int64_t)P.cnt[(int64_t)(b + 1) * P.n_blk] : (int64_t)*total;
            v = (int32_t)std::max<int64_t>(1, (end - start + kReducePart - 1) / kReducePart);
        }
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int32_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (b < P.n_buckets) parts[b] = carry + sh[threadIdx.x] - v;
        carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[P.n_buckets] = carry;
}

// Entries per reduction window: the window's FD 64-bit sums fill 64 or 48 KiB of LDS.
template <int FD> constexpr int kLog2Window = FD == 2 ? 12 : 11;

// Block (i, w): part i of the work list, window w (2^kLog2Window entries) of its bucket.  A
// bucket cut into one part is added to the table gradient directly; parts of a bucket cut into
// several add their nonzero window entries with atomics.
// The window is summed in 64-bit fixed point with integer LDS atomics (several times the rate
// of floating-point LDS atomics): with |value| < 2^e over the round and at most N additions,
// the scale 2^s, s = 62 - e - ceil(log2 N), keeps every partial sum below 2^62 while the unit
// is 2^-31 to 2^-32 of the largest addition (2^18 samples per round); the sum is exact in
// that unit and independent of order.
template <int FD>
__global__ void __launch_bounds__(256) k_enc_bwd_reduce(EncBwdParams P, const int32_t* __restrict__ total,
                                                        const int32_t* __restrict__ parts) {
    constexpr int LW = kLog2Window<FD>, WN = 1 << LW;
    __shared__ unsigned long long s_acc[FD * WN];
    const int i = blockIdx.x, w = blockIdx.y;
    if (i >= parts[P.n_buckets]) return;
    int lo = 0, hi = P.n_buckets - 1;                    // bucket b: parts[b] <= i < parts[b + 1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (parts[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const int b = lo;
    const int n_parts = parts[b + 1] - parts[b], part = i - parts[b];
    const int wn = P.SB < LW ? (1 << P.SB) : WN;     // entries per window
    for (int k = threadIdx.x; k < FD * wn; k += 256) s_acc[k] = 0ull;
    const float vmax = __uint_as_float(*P.vmax);
    const bool finite = isfinite(vmax);
    int ev = 0;
    if (vmax > 0.f && finite) (void)frexpf(vmax, &ev);          // vmax < 2^ev
    int nb = 0;
    while (nb < 40 && ((int64_t)1 << nb) < (int64_t)*total + 1) ++nb;
    const int sc = 62 - ev - nb;
    __syncthreads();
    const int64_t b_start = P.cnt[(int64_t)b * P.n_blk];
    const int64_t b_end = b + 1 < P.n_buckets ? (int64_t)P.cnt[(int64_t)(b + 1) * P.n_blk] : (int64_t)*total;
    const int64_t start = b_start + (int64_t)part * kReducePart;
    const int64_t end = std::min<int64_t>(b_end, start + kReducePart);
    // Thread t takes 16 consecutive records per step (16-byte loads, coalesced across the
    // wave): records next to each other come from neighbouring samples and often hit the same
    // entries, so runs of equal keys are summed in registers before the LDS atomics, and the
    // lanes of a wave work 16 records apart.  Every record adds at most |a| < 2^e in all (its
    // two parts split a by weights summing to 1), so N counts records in the scale above.
    const int64_t g0 = start >> 4, g1 = (end + 15) >> 4;      // aligned groups of 16
    auto add_fixed = [&](uint32_t e, const float* r) {       // e: entry within the bucket
        if ((int)(e >> LW) != w) return;
        const int k = (int)(e & (WN - 1));
#pragma unroll
        for (int f = 0; f < FD; ++f)
            if (r[f] != 0.f) atomicAdd(&s_acc[FD * k + f], (unsigned long long)llrint(ldexp((double)r[f], sc)));
    };
    for (int64_t g = g0 + threadIdx.x; g < g1; g += 256) {
        const int64_t base = g << 4;
        float vv[16 * kRecFloats];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float4 t = *reinterpret_cast<const float4*>(P.val + (base + r) * kRecFloats);
            vv[4 * r] = t.x; vv[4 * r + 1] = t.y; vv[4 * r + 2] = t.z; vv[4 * r + 3] = t.w;
        }
        bool have = false;
        uint32_t cur = 0;
        float r0[FD], r1[FD];
#pragma unroll
        for (int f = 0; f < FD; ++f) r0[f] = r1[f] = 0.f;
        auto flush = [&]() {
            if (!have) return;
            if constexpr (FD == 2) {
                add_fixed(cur & 0xffffu, r0);
                add_fixed(cur >> 16, r1);
            } else {
                add_fixed(cur, r0);
            }
        };
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t k = base + r;
            if (k < start || k >= end) continue;
            const float* rec = vv + kRecFloats * r;
            const uint32_t key = __float_as_uint(rec[3]);
            float c0[FD], c1[FD];
            if constexpr (FD == 2) {
                const float wx = rec[2];
                const float wl = 1.f - wx;
#pragma unroll
                for (int f = 0; f < FD; ++f) { c0[f] = wl * rec[f]; c1[f] = wx * rec[f]; }
            } else {
#pragma unroll
                for (int f = 0; f < FD; ++f) { c0[f] = rec[f]; c1[f] = 0.f; }
            }
            if (!have || key != cur) {
                flush();
                have = true;
                cur = key;
#pragma unroll
                for (int f = 0; f < FD; ++f) { r0[f] = c0[f]; r1[f] = c1[f]; }
            } else {
#pragma unroll
                for (int f = 0; f < FD; ++f) { r0[f] += c0[f]; r1[f] += c1[f]; }
            }
        }
        flush();
    }
    __syncthreads();
    const int l = b / P.NBL, slice = b % P.NBL;
    float* g = P.g_tables + (((size_t)l << P.enc.log2T) + ((size_t)slice << P.SB) + ((size_t)w << LW)) * FD;
    // a non-finite addition poisons the window, so the step's finiteness check skips the update
    auto value = [&](int k) { return finite ? (float)ldexp((double)(long long)s_acc[k], -sc) : NAN; };
    if (n_parts == 1) {
        for (int k = threadIdx.x; k < FD * wn; k += 256) g[k] += value(k);
    } else {
        for (int k = threadIdx.x; k < FD * wn; k += 256)
            if (s_acc[k] != 0ull || !finite) unsafeAtomicAdd(&g[k], value(k));
    }
}

// ------------------------------------------------------------------ the loss on its own
// nif_loss uses the upper halves of the model's accumulators (sums at dacc[9..13], scale 1 at
// dacc[15], positives at tcount[8]), so a training step's loss scale and counters are untouched.
constexpr int kLossDacc = 9, kLossTcount = 8;

__global__ void k_loss_begin(double* dacc, int64_t* tcount) {
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 5; ++k) dacc[DA_SUM + k] = 0.0;
    dacc[DA_SCALE_USED] = 1.0;
    tcount[TC_NPOS] = 0;
}

// Task losses and total (Eq. of the uncertainty-weighted loss) and d total / d s.
__global__ void k_loss_out(const double* dacc, const int64_t* tcount, const float* s, int64_t B, int fixed,
                           float* losses, float* g_s) {
    if (threadIdx.x != 0) return;
    const double P = (double)tcount[TC_NPOS];
    double total = 0.0;
    for (int k = 0; k < 5; ++k) {
        const double Lk = k == 0 ? dacc[DA_SUM] / (double)B : (P > 0 ? dacc[DA_SUM + k] / P : 0.0);
        const double w = (k == 0 || k == 4 ? 1.0 : 0.5) * exp(-(double)s[k]);
        losses[k] = (float)Lk;
        if (fixed) {
            total += Lk;
            if (g_s) g_s[k] = 0.f;
        } else {
            total += w * Lk + 0.5 * s[k];
            if (g_s) g_s[k] = (float)(-w * Lk + 0.5);
        }
    }
    losses[5] = (float)total;
}


// ------------------------------------------------------------------ step bookkeeping

__global__ void k_check_finite(const float* __restrict__ a, int64_t n, int64_t* tcount) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(a[i]);
    if (__ballot(bad) && lane_id() == 0) tcount[TC_NONFINITE] = 1;
}

// Losses, d total / d s, dynamic loss scale, skip decision, Adam bias corrections (one thread).
__global__ void k_finalize(double* dacc, int64_t* tcount, const float* s, float* g_s, float* losses, int64_t B,
                           int dynamic, int grow_interval, float beta1, float beta2, int fixed) {
    if (threadIdx.x != 0) return;
    const double P = (double)tcount[TC_NPOS];
    double Ls[5], w[5];
    Ls[0] = dacc[DA_SUM] / (double)B;
    for (int k = 1; k < 5; ++k) Ls[k] = P > 0 ? dacc[DA_SUM + k] / P : 0.0;
    w[0] = exp(-(double)s[0]); w[1] = 0.5 * exp(-(double)s[1]); w[2] = 0.5 * exp(-(double)s[2]);
    w[3] = 0.5 * exp(-(double)s[3]); w[4] = exp(-(double)s[4]);
    double total = 0.0;
    for (int k = 0; k < 5; ++k) {
        if (fixed) {                       // plain sum; s is neither used nor trained
            total += Ls[k];
            g_s[k] = 0.f;
        } else {
            total += w[k] * Ls[k] + 0.5 * s[k];
            g_s[k] = (float)(-w[k] * Ls[k] + 0.5);
        }
        losses[k] = (float)Ls[k];
        losses[6 + k] = s[k];
    }
    losses[5] = (float)total;
    const bool bad = tcount[TC_NONFINITE] != 0 || !isfinite(total);
    double scale = dacc[DA_SCALE];
    losses[11] = (float)dacc[DA_SCALE_USED];
    if (bad) {
        tcount[TC_SKIP] = 1;
        tcount[TC_GOOD] = 0;
        if (dynamic) scale = fmax(scale * 0.5, 1.0 / 65536.0);
    } else {
        tcount[TC_SKIP] = 0;
        tcount[TC_STEP] += 1;
        tcount[TC_GOOD] += 1;
        if (dynamic && tcount[TC_GOOD] >= grow_interval) { scale *= 2.0; tcount[TC_GOOD] = 0; }
    }
    dacc[DA_SCALE] = scale;
    const double t = (double)tcount[TC_STEP];
    dacc[DA_C1] = 1.0 - pow((double)beta1, t);
    dacc[DA_C2] = 1.0 - pow((double)beta2, t);
    losses[12] = bad ? 1.f : 0.f;
    losses[13] = (float)P;
    losses[14] = 0.f;
    losses[15] = 0.f;
}

struct AdamParams {
    float *tables, *g_tables, *m_tables, *v_tables;
    __half* tables_h;
    float *mlp, *g_mlp, *m_mlp, *v_mlp;
    float *s, *g_s, *m_s, *v_s;
    int64_t n_table, n_mlp;
    float lr_table, lr_mlp, lr_s, beta1, beta2, eps;
};

__device__ __forceinline__ float adam_one(float& th, float g, float& m, float& v, float lr, float b1, float b2,
                                          float eps, float c1, float c2) {
    m = b1 * m + (1.f - b1) * g;
    v = b2 * v + (1.f - b2) * g * g;
    const float mh = m / c1, vh = v / c2;
    th -= lr * mh / (sqrtf(vh) + eps);
    return th;
}

__global__ void k_adam(AdamParams A, const double* __restrict__ dacc, const int64_t* __restrict__ tcount) {
    if (tcount[TC_SKIP]) return;
    const float inv = (float)(1.0 / dacc[DA_SCALE_USED]);
    const float c1 = (float)dacc[DA_C1], c2 = (float)dacc[DA_C2];
    const int64_t n = A.n_table + A.n_mlp + 5;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < A.n_table) {
            float th = A.tables[i], m = A.m_tables[i], v = A.v_tables[i];
            adam_one(th, A.g_tables[i] * inv, m, v, A.lr_table, A.beta1, A.beta2, A.eps, c1, c2);
            A.tables[i] = th; A.m_tables[i] = m; A.v_tables[i] = v;
            if (A.tables_h) A.tables_h[i] = __float2half_rn(th);
        } else if (i < A.n_table + A.n_mlp) {
            const int64_t k = i - A.n_table;
            float th = A.mlp[k], m = A.m_mlp[k], v = A.v_mlp[k];
            adam_one(th, A.g_mlp[k] * inv, m, v, A.lr_mlp, A.beta1, A.beta2, A.eps, c1, c2);
            A.mlp[k] = th; A.m_mlp[k] = m; A.v_mlp[k] = v;
        } else {
            const int64_t k = i - A.n_table - A.n_mlp;
            float th = A.s[k], m = A.m_s[k], v = A.v_s[k];
            adam_one(th, A.g_s[k], m, v, A.lr_s, A.beta1, A.beta2, A.eps, c1, c2);
            A.s[k] = th; A.m_s[k] = m; A.v_s[k] = v;
        }
    }
}

// ------------------------------------------------------------------ host launchers

static int cus() {
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
    }
    return n;
}

static unsigned grid_for(int64_t n, int per = 256, int64_t cap_per_cu = 8) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, cus() * cap_per_cu));
}

template <int HW, int PREC>
static void launch_mlp_bwd(const BwdParams& bp, const float* dz, const float* acts, float* delta, int64_t B, hipStream_t st) {
    constexpr int CB = HW >= 128 ? 2 : 4;
    const int64_t tiles = (B + 16 * CB - 1) / (16 * CB);
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, cus() * 8));
    hipLaunchKernelGGL((k_mlp_bwd<HW, PREC>), dim3(blocks), dim3(256), 0, st, bp, dz, acts, delta, B);
}

template <int PREC>
static int dispatch_mlp_bwd(int hw, const BwdParams& bp, const float* dz, const float* acts, float* delta, int64_t B,
                            hipStream_t st) {
    switch (hw) {
        case 16: launch_mlp_bwd<16, PREC>(bp, dz, acts, delta, B, st); break;
        case 32: launch_mlp_bwd<32, PREC>(bp, dz, acts, delta, B, st); break;
        case 64: launch_mlp_bwd<64, PREC>(bp, dz, acts, delta, B, st); break;
        case 128: launch_mlp_bwd<128, PREC>(bp, dz, acts, delta, B, st); break;
        default: return fail(NIF_E_UNSUPPORTED, "hidden_width must be 16, 32, 64 or 128");
    }
    return NIF_OK;
}

// Backward from dz (already in m->dz) to the gradient accumulators; activations in m->acts.
// One layer's weight gradient over rows [0, B) of d (stride dstride) and h (stride hstride),
// added to gW / gb: K-sliced MFMA partials, then a sum per output.
template <int PREC>
static void launch_dw_part(const DwArgs& A, dim3 grid, hipStream_t st) {
    switch (A.M_pad / 16) {
        case 1: hipLaunchKernelGGL((k_dw_part<1, PREC>), grid, dim3(256), 0, st, A); break;
        case 2: hipLaunchKernelGGL((k_dw_part<2, PREC>), grid, dim3(256), 0, st, A); break;
        case 4: hipLaunchKernelGGL((k_dw_part<4, PREC>), grid, dim3(256), 0, st, A); break;
        default: hipLaunchKernelGGL((k_dw_part<8, PREC>), grid, dim3(256), 0, st, A); break;
    }
}

// Weight gradient of one layer; with BF16/FP16 MLP arithmetic its operands are rounded to that
// precision as in the forward and the MLP backward (FP32 accumulation either way).
template <int PREC>
static void launch_dw_tile(const DwArgs& A, dim3 grid, hipStream_t st) {
    if (A.M_pad == 128) hipLaunchKernelGGL((k_dw_tile<2, 2, PREC>), grid, dim3(256), 0, st, A);
    else hipLaunchKernelGGL((k_dw_tile<1, 4, PREC>), grid, dim3(256), 0, st, A);
}

static int weight_grad(nif_model* m, int layer, const float* d, int dstride, int M_pad, const float* h, int64_t B,
                       int cus, int32_t precision, hipStream_t st) {
    const int N = m->dims[layer];
    if (dw_tiled(M_pad, N) && dstride % 4 == 0) {
        DwArgs A = dw_tile_shape(M_pad, N, B, cus);
        A.d = d;
        A.dstride = dstride;
        A.M_real = m->dims[layer + 1];
        A.h = h;
        A.hstride = N;
        A.part = m->dw_part;
        if (dw_part_floats(A) > m->dw_part_n) return fail(NIF_E_STATE, "weight-gradient scratch too small");
        const int ct = dw_tile_ct(M_pad);
        const dim3 grid((unsigned)A.n_slots, (unsigned)((A.n_cb + ct - 1) / ct));
        if (precision == NIF_PREC_BF16) launch_dw_tile<P_BF16>(A, grid, st);
        else if (precision == NIF_PREC_FP16) launch_dw_tile<P_FP16>(A, grid, st);
        else launch_dw_tile<P_FP32>(A, grid, st);
        const int64_t n_out = (int64_t)A.M_real * A.N + A.M_real;
        hipLaunchKernelGGL(k_dw_sum, dim3((unsigned)((n_out + 63) / 64)), dim3(64 * kDwSumGroups), 0, st, A,
                           m->g_mlp + m->w_off[layer], A.N, m->g_mlp + m->b_off[layer]);
        return NIF_OK;
    }
    DwArgs A = dw_shape(M_pad, N, B, cus);
    A.d = d;
    A.dstride = dstride;
    A.M_real = m->dims[layer + 1];
    A.h = h;
    A.hstride = m->dims[layer];
    A.part = m->dw_part;
    if (dw_part_floats(A) > m->dw_part_n) return fail(NIF_E_STATE, "weight-gradient scratch too small");
    const dim3 grid((unsigned)((B + A.Kc - 1) / A.Kc), (unsigned)(A.ks > 1 ? 1 : (A.n_cb + 3) / 4));
    if (precision == NIF_PREC_BF16) launch_dw_part<P_BF16>(A, grid, st);
    else if (precision == NIF_PREC_FP16) launch_dw_part<P_FP16>(A, grid, st);
    else launch_dw_part<P_FP32>(A, grid, st);
    const int64_t n_out = (int64_t)A.M_real * A.N + A.M_real;
    hipLaunchKernelGGL(k_dw_sum, dim3((unsigned)((n_out + 63) / 64)), dim3(64 * kDwSumGroups), 0, st, A,
                       m->g_mlp + m->w_off[layer], A.N, m->g_mlp + m->b_off[layer]);
    return NIF_OK;
}

// Table-gradient parameters of a batch (points SoA with stride B, delta rows from drow0).
static EncBwdParams table_grad_params(nif_model* m, const float* x0, const float* x1, int64_t B, float* dx0, float* dx1) {
    EncBwdParams ep;
    memset(&ep, 0, sizeof(ep));
    ep.enc = make_net_params(m, NIF_PREC_FP32).enc;
    ep.W0t = m->mlp_pad_f32 + m->wt_off[0];
    ep.delta0 = m->delta;
    ep.drow0 = 0;
    ep.x0 = x0; ep.x1 = x1;
    ep.HW = m->desc.hidden_width; ep.E = m->E; ep.S = m->S;
    ep.g_tables = m->g_tables;
    ep.dx0 = dx0; ep.dx1 = dx1;
    ep.B = B;
    const int log2T = m->desc.log2_table;
    ep.SB = log2T <= 12 ? log2T : std::max(12, log2T - 8);
    ep.NBL = 1 << (log2T - ep.SB);
    const int n_sets = m->desc.per_sample_tables ? m->S : 1;
    ep.n_buckets = m->desc.levels * n_sets * ep.NBL;
    ep.cnt = m->bwd_cnt; ep.val = m->bwd_val;
    ep.cap = m->bwd_round * 2 * m->S * m->desc.levels * 8;
    ep.vmax = nullptr;
    return ep;
}

// A round of the table gradient over samples [c0, c0 + n), n <= bwd_round, on stream sd: the
// count and scan (positions only) when it begins, one fill launch per chunk once the chunk's
// first-layer deltas exist, then the parts and the reduction.  Rounds share their scratch, so
// they run in stream order.
struct TgRound {
    EncBwdParams ep;
    int32_t* total;
    int32_t* parts;
};

template <int FD>
static TgRound tg_begin_fd(nif_model* m, EncBwdParams ep, int64_t c0, int64_t n, hipStream_t sd) {
    constexpr int LG = kLevelGroup<FD>;
    ep.c0 = c0;
    ep.n = n;
    ep.blk0 = 0;
    const int64_t n_tiles = (ep.n + 15) / 16;
    ep.n_blk = (int32_t)((n_tiles + kBwdTilesPerBlock - 1) / kBwdTilesPerBlock);
    const int64_t n_cnt = (int64_t)ep.n_buckets * ep.n_blk;
    const int n_chunks = (int)((n_cnt + 4095) / 4096);
    int32_t* sums = m->bwd_scan;
    TgRound R;
    R.total = m->bwd_scan + n_chunks;
    R.parts = R.total + 1;
    ep.vmax = reinterpret_cast<uint32_t*>(R.parts + ep.n_buckets + 1);
    const int n_sets = m->desc.per_sample_tables ? m->S : 1;
    const dim3 fg((unsigned)ep.n_blk, (unsigned)(m->desc.levels / LG));
    const size_t lds_f = sizeof(int32_t) * LG * (size_t)ep.NBL * n_sets;
    hipLaunchKernelGGL(k_enc_bwd_count<FD>, fg, dim3(256), lds_f, sd, ep);
    hipLaunchKernelGGL(k_scan_sums, dim3(n_chunks), dim3(256), 0, sd, ep.cnt, n_cnt, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, sd, sums, n_chunks, R.total);
    hipLaunchKernelGGL(k_scan_apply, dim3(n_chunks), dim3(256), 0, sd, ep.cnt, n_cnt, sums);
    R.ep = ep;
    return R;
}

// Fill of the round's samples [c0, c0 + n) (whole blocks of the round: c0 - round start is a
// multiple of 16 kBwdTilesPerBlock, or n reaches the round's end); delta rows of sample seg at
// delta + (seg - drow0) HW.
template <int FD>
static void tg_fill_fd(nif_model* m, const TgRound& R, const float* delta, int64_t drow0, int64_t c0, int64_t n,
                       hipStream_t sd) {
    constexpr int LG = kLevelGroup<FD>;
    EncBwdParams ep = R.ep;
    ep.delta0 = delta;
    ep.drow0 = drow0;
    const int64_t per_blk = 16 * kBwdTilesPerBlock;
    ep.blk0 = (int32_t)((c0 - ep.c0) / per_blk);
    const int64_t blk1 = std::min<int64_t>(ep.n_blk, (c0 + n - ep.c0 + per_blk - 1) / per_blk);
    const int hw = m->desc.hidden_width;
    const int n_sets = m->desc.per_sample_tables ? m->S : 1;
    const dim3 fg((unsigned)(blk1 - ep.blk0), (unsigned)(m->desc.levels / LG));
    // the fill's staged first-layer rows: 4 per PE combination, hw + 4 floats each (up to 60 KiB)
    const int nloc = LG * ep.NBL * n_sets;
    const size_t lds_f = sizeof(int32_t) * (size_t)nloc;
    const size_t w_bytes = sizeof(float) * 4 * (size_t)(2 * m->S) * (size_t)(hw + 4);
    const size_t cur_bytes = sizeof(int32_t) * (size_t)((nloc + 3) & ~3);
    ep.w_lds = cur_bytes + w_bytes <= kFillLdsMax ? 1 : 0;
    const size_t lds_fill = ep.w_lds ? cur_bytes + w_bytes : lds_f;
    switch (hw) {
        case 16: hipLaunchKernelGGL((k_enc_bwd_fill<16, FD>), fg, dim3(256), lds_fill, sd, ep); break;
        case 32: hipLaunchKernelGGL((k_enc_bwd_fill<32, FD>), fg, dim3(256), lds_fill, sd, ep); break;
        case 64: hipLaunchKernelGGL((k_enc_bwd_fill<64, FD>), fg, dim3(256), lds_fill, sd, ep); break;
        default: hipLaunchKernelGGL((k_enc_bwd_fill<128, FD>), fg, dim3(256), lds_fill, sd, ep); break;
    }
}

template <int FD>
static void tg_end_fd(nif_model* m, const TgRound& R, hipStream_t sd) {
    constexpr int LW = kLog2Window<FD>;
    const EncBwdParams& ep = R.ep;
    const unsigned n_win = ep.SB > LW ? 1u << (ep.SB - LW) : 1u;
    hipLaunchKernelGGL(k_enc_bwd_parts, dim3(1), dim3(1024), 0, sd, ep, R.total, R.parts);
    const int64_t max_parts = ep.n_buckets + (ep.n * 2 * m->S * m->desc.levels * 8) / kReducePart + 1;
    hipLaunchKernelGGL(k_enc_bwd_reduce<FD>, dim3((unsigned)max_parts, n_win), dim3(256), 0, sd, ep, R.total, R.parts);
}

static TgRound tg_begin(nif_model* m, const EncBwdParams& ep, int64_t c0, int64_t n, hipStream_t sd) {
    return m->desc.feat_dim == 3 ? tg_begin_fd<3>(m, ep, c0, n, sd) : tg_begin_fd<2>(m, ep, c0, n, sd);
}
static void tg_fill(nif_model* m, const TgRound& R, const float* delta, int64_t drow0, int64_t c0, int64_t n,
                    hipStream_t sd) {
    if (m->desc.feat_dim == 3) tg_fill_fd<3>(m, R, delta, drow0, c0, n, sd);
    else tg_fill_fd<2>(m, R, delta, drow0, c0, n, sd);
}
static void tg_end(nif_model* m, const TgRound& R, hipStream_t sd) {
    if (m->desc.feat_dim == 3) tg_end_fd<3>(m, R, sd);
    else tg_end_fd<2>(m, R, sd);
}

// Backward from m->dz.  enc_stored: the forward's encoding [B][E], or null to recompute it
// per chunk of bwd_chunk samples for the first layer's weight gradient.
static int backward_core(nif_model* m, const float* x0, const float* x1, int64_t B, float* dx0, float* dx1,
                         int32_t precision, const float* enc_stored, hipStream_t st) {
    const int hw = m->desc.hidden_width, nh = m->desc.hidden_layers;
    BwdParams bp;
    memset(&bp, 0, sizeof(bp));
    bp.n_hidden = nh;
    for (int i = 1; i < m->n_layers; ++i) {
        if (precision == NIF_PREC_FP32) bp.Wt[i] = m->mlp_pad_f32 + m->wt_off[i];
        else if (precision == NIF_PREC_BF16) bp.Wt[i] = m->mlp_pad_bf16 + m->wt_off[i];
        else bp.Wt[i] = m->mlp_pad_f16 + m->wt_off[i];
    }
    int rc;
    if (precision == NIF_PREC_FP32) rc = dispatch_mlp_bwd<P_FP32>(hw, bp, m->dz, m->acts, m->delta, B, st);
    else if (precision == NIF_PREC_BF16) rc = dispatch_mlp_bwd<P_BF16>(hw, bp, m->dz, m->acts, m->delta, B, st);
    else rc = dispatch_mlp_bwd<P_FP16>(hw, bp, m->dz, m->acts, m->delta, B, st);
    if (rc) return rc;
    // Fork: the table-gradient chain (reads delta[0], x0, x1; writes the table gradient and, by
    // atomics, dx0 / dx1) runs on the model's side stream while this stream forms the weight
    // gradients (reads the deltas, activations and the encoding; writes the MLP gradient); the
    // two touch disjoint scratch.
    hipStream_t sd = m->side;
    if ((rc = check_hip(hipEventRecord(m->ev_fork, st), "backward fork"))) return rc;
    if ((rc = check_hip(hipStreamWaitEvent(sd, m->ev_fork, 0), "backward fork"))) return rc;
    // encoding backward (layer 0): count / scan / fill / reduce per round of samples
    const EncBwdParams ep = table_grad_params(m, x0, x1, B, dx0, dx1);
    for (int64_t c0 = 0; c0 < B; c0 += m->bwd_round) {
        const int64_t n = std::min<int64_t>(m->bwd_round, B - c0);
        const TgRound R = tg_begin(m, ep, c0, n, sd);
        tg_fill(m, R, m->delta, 0, c0, n, sd);
        tg_end(m, R, sd);
    }
    if ((rc = check_hip(hipEventRecord(m->ev_join, sd), "backward join"))) return rc;
    // weight gradients of every layer (layer 0 from the stored or the recomputed encoding)
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    for (int i = 0; i < m->n_layers; ++i) {
        const bool out = i == m->n_layers - 1;
        const float* d = out ? m->dz : m->delta + (size_t)i * B * hw;
        const int ds = out ? 16 : hw;
        if (rc) break;
        if (i > 0) {
            rc = weight_grad(m, i, d, ds, ds, m->acts + (size_t)(i - 1) * B * hw, B, cus, precision, st);
        } else if (enc_stored) {
            rc = weight_grad(m, 0, d, ds, ds, enc_stored, B, cus, precision, st);
        } else {
            for (int64_t c0 = 0; c0 < B && !rc; c0 += m->bwd_chunk) {
                const int64_t n = std::min<int64_t>(m->bwd_chunk, B - c0);
                if (!(rc = encode_pairs_launch(m, x0 + c0, x1 + c0, n, B, precision, m->enc, st)))
                    rc = weight_grad(m, 0, d + (size_t)c0 * ds, ds, ds, m->enc, n, cus, precision, st);
            }
        }
    }
    // join before anything that reads the table gradient or dx
    const int rc_join = check_hip(hipStreamWaitEvent(st, m->ev_join, 0), "backward join");
    if (rc) return rc;
    if (rc_join) return rc_join;
    if (dx0 && m->GW > 0) {                  // concatenated encoding: d x through the raw gamma values
        const int E_phi = 2 * m->S * m->desc.levels * m->desc.feat_dim;
        hipLaunchKernelGGL(k_gamma_dx, dim3(grid_for(B)), dim3(256), 0, st, m->mlp_pad_f32 + m->wt_off[0], m->delta,
                           hw, E_phi, m->GW, x0, x1, B, dx0, dx1);
    }
    return check_hip(hipGetLastError(), "backward launch");
}

// Zero the gradient accumulators with kernels (no memset nodes when the caller captures a graph).
int zero_grads_launch(nif_model* m, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(m->n_table)), dim3(256), 0, st, m->g_tables, m->n_table);
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(m->n_mlp)), dim3(256), 0, st, m->g_mlp, m->n_mlp);
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(256), 0, st, m->g_s, (int64_t)8);
    return check_hip(hipGetLastError(), "zero grads");
}

int backward_launch(nif_model* m, const float* x0, const float* x1, int64_t B, const float* dh, int32_t, float* dx0,
                    float* dx1, int32_t precision, hipStream_t st) {
    if (B == 0) return NIF_OK;
    int rc = forward_launch(m, x0, x1, B, m->zbuf, precision, m->acts, nullptr, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pad_dz, dim3(grid_for(B * 16)), dim3(256), 0, st, dh, m->H, B, m->dz);
    if (dx0) hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(3 * B)), dim3(256), 0, st, dx0, 3 * B);
    if (dx1) hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(3 * B)), dim3(256), 0, st, dx1, 3 * B);
    return backward_core(m, x0, x1, B, dx0, dx1, precision, nullptr, st);
}

int loss_launch(nif_model* m, const float* heads, int64_t B, const nif_batch* b, const float* s, int32_t fixed,
                float* losses, float* d_heads, float* d_s, hipStream_t st) {
    double* dacc = m->dacc + kLossDacc;
    int64_t* tcount = m->tcount + kLossTcount;
    hipLaunchKernelGGL(k_loss_begin, dim3(1), dim3(64), 0, st, dacc, tcount);
    hipLaunchKernelGGL(k_count_pos, dim3(grid_for(B)), dim3(256), 0, st, b->hit, B, tcount);
    hipLaunchKernelGGL(k_loss, dim3(grid_for(B)), dim3(256), 0, st, heads, m->H, B, B, B, b->hit, b->t, b->n, b->a,
                       b->m, s, tcount, dacc, d_heads, m->H, b->x0, b->x1, m->desc.dist_head, fixed);
    hipLaunchKernelGGL(k_loss_out, dim3(1), dim3(64), 0, st, dacc, tcount, s, B, fixed, losses, d_s);
    return check_hip(hipGetLastError(), "loss launch");
}

// Batches at least this large are put in spatial order before the step (nif_order.hip).
constexpr int64_t kOrderMinBatch = 1 << 14;

int train_step_launch(nif_model* m, const nif_batch* b_in, int64_t B, const nif_train_cfg* cfg, float* losses,
                      hipStream_t st) {
    nif_batch ordered;
    const nif_batch* b = b_in;
    if (B >= kOrderMinBatch) {
        const int rc = order_batch(m, b_in, B, &ordered, st);
        if (rc) return rc;
        b = &ordered;
    }
    const int prec = cfg->precision;
    const float scale_init = cfg->loss_scale_init > 0.f ? cfg->loss_scale_init : (prec == NIF_PREC_FP16 ? 32768.f : 1.f);
    if (cfg->store_encoding && !m->enc_all)
        return fail(NIF_E_STATE, "store_encoding needs nif_model_reserve_encoding first");
    hipLaunchKernelGGL(k_train_begin, dim3(1), dim3(64), 0, st, m->dacc, m->tcount, scale_init);
    hipLaunchKernelGGL(k_count_pos, dim3(grid_for(B)), dim3(256), 0, st, b->hit, B, m->tcount);
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(m->n_table)), dim3(256), 0, st, m->g_tables, m->n_table);
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(m->n_mlp)), dim3(256), 0, st, m->g_mlp, m->n_mlp);
    // The step runs per chunk of bwd_chunk samples: forward, loss rows (the means use the whole
    // batch's size and positive count, known before), MLP backward; then the chunk's table
    // gradient goes to the side stream while this stream forms its weight gradients (the first
    // layer's from the encoding, recomputed unless stored) and moves on to the next chunk.
    // Chunk c keeps its heads, d heads, activations and deltas in rows of its own block of the
    // batch-sized buffers, so the side stream can still read chunk c's deltas meanwhile.
    const int hw = m->desc.hidden_width, nh = m->desc.hidden_layers, H = m->H;
    BwdParams bp;
    memset(&bp, 0, sizeof(bp));
    bp.n_hidden = nh;
    for (int i = 1; i < m->n_layers; ++i) {
        if (prec == NIF_PREC_FP32) bp.Wt[i] = m->mlp_pad_f32 + m->wt_off[i];
        else if (prec == NIF_PREC_BF16) bp.Wt[i] = m->mlp_pad_bf16 + m->wt_off[i];
        else bp.Wt[i] = m->mlp_pad_f16 + m->wt_off[i];
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    EncBwdParams ep = table_grad_params(m, b->x0, b->x1, B, nullptr, nullptr);
    hipStream_t sd = m->side;
    int rc = NIF_OK;
    bool forked = false;
    // weight gradients of the chunk at rows [c0, c0 + n)
    auto chunk_weight_grads = [&](int64_t c0, int64_t n) {
        float* acts_c = m->acts + (size_t)c0 * nh * hw;
        float* delta_c = m->delta + (size_t)c0 * nh * hw;
        float* dz_c = m->dz + (size_t)c0 * 16;
        float* enc_c = cfg->store_encoding ? m->enc_all + (size_t)c0 * m->E : nullptr;
        int r = NIF_OK;
        for (int i = 0; i < m->n_layers && !r; ++i) {
            const bool out = i == m->n_layers - 1;
            const float* d = out ? dz_c : delta_c + (size_t)i * n * hw;
            const int ds = out ? 16 : hw;
            if (i > 0) {
                r = weight_grad(m, i, d, ds, ds, acts_c + (size_t)(i - 1) * n * hw, n, cus, prec, st);
            } else if (enc_c) {
                r = weight_grad(m, 0, d, ds, ds, enc_c, n, cus, prec, st);
            } else if (!(r = encode_pairs_launch(m, b->x0 + c0, b->x1 + c0, n, B, prec, m->enc, st))) {
                r = weight_grad(m, 0, d, ds, ds, m->enc, n, cus, prec, st);
            }
        }
        return r;
    };
    // The weight gradients of chunk c are issued after chunk c + 1's MLP backward, so the next
    // fill (the longer branch) can start as early as possible.  A table-gradient round (up to
    // bwd_round samples, whole chunks) counts and scans its additions as soon as it begins (the
    // positions are known), fills once per chunk after that chunk's MLP backward, and reduces
    // after its last chunk.
    int64_t prev_c0 = -1, prev_n = 0;
    int64_t round_end = 0;
    TgRound R;
    memset(&R, 0, sizeof(R));
    bool round_open = false;
    for (int64_t c0 = 0; c0 < B && !rc; c0 += m->bwd_chunk) {
        const int64_t n = std::min<int64_t>(m->bwd_chunk, B - c0);
        float* acts_c = m->acts + (size_t)c0 * nh * hw;      // [hidden layers][n][hw]
        float* delta_c = m->delta + (size_t)c0 * nh * hw;
        float* z_c = m->zbuf + (size_t)c0 * H;
        float* dz_c = m->dz + (size_t)c0 * 16;
        float* enc_c = cfg->store_encoding ? m->enc_all + (size_t)c0 * m->E : nullptr;
        if (c0 >= round_end) {                  // a round begins with this chunk
            if (round_open) tg_end(m, R, sd);
            const int64_t rn = std::min<int64_t>(m->bwd_round, B - c0);
            if ((rc = check_hip(hipEventRecord(m->ev_fork, st), "train fork"))) break;
            if ((rc = check_hip(hipStreamWaitEvent(sd, m->ev_fork, 0), "train fork"))) break;
            forked = true;
            R = tg_begin(m, ep, c0, rn, sd);
            round_open = true;
            round_end = c0 + rn;
        }
        if ((rc = forward_rows_launch(m, b->x0 + c0, b->x1 + c0, n, B, z_c, prec, acts_c, enc_c, st))) break;
        hipLaunchKernelGGL(k_loss, dim3(grid_for(n)), dim3(256), 0, st, z_c, H, n, B, B, b->hit + c0, b->t + c0,
                           b->n + c0, b->a + c0, b->m + c0, m->s, m->tcount, m->dacc, dz_c, 16, b->x0 + c0, b->x1 + c0,
                           m->desc.dist_head, cfg->fixed_task_weights);
        if (prec == NIF_PREC_FP32) rc = dispatch_mlp_bwd<P_FP32>(hw, bp, dz_c, acts_c, delta_c, n, st);
        else if (prec == NIF_PREC_BF16) rc = dispatch_mlp_bwd<P_BF16>(hw, bp, dz_c, acts_c, delta_c, n, st);
        else rc = dispatch_mlp_bwd<P_FP16>(hw, bp, dz_c, acts_c, delta_c, n, st);
        if (rc) break;
        if ((rc = check_hip(hipEventRecord(m->ev_fork, st), "train fork"))) break;
        if ((rc = check_hip(hipStreamWaitEvent(sd, m->ev_fork, 0), "train fork"))) break;
        tg_fill(m, R, delta_c, c0, c0, n, sd);     // layer 0 of the chunk's block
        if (prev_c0 >= 0 && (rc = chunk_weight_grads(prev_c0, prev_n))) break;
        prev_c0 = c0;
        prev_n = n;
    }
    if (!rc && round_open) tg_end(m, R, sd);
    if (!rc && prev_c0 >= 0) rc = chunk_weight_grads(prev_c0, prev_n);
    if (forked) {                               // join before the gradients are read
        const int rj = check_hip(hipEventRecord(m->ev_join, sd), "train join");
        const int rw = rj ? rj : check_hip(hipStreamWaitEvent(st, m->ev_join, 0), "train join");
        if (!rc) rc = rw;
    }
    if (rc) return rc;
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(m->n_table)), dim3(256), 0, st, m->g_tables, m->n_table, m->tcount);
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(m->n_mlp)), dim3(256), 0, st, m->g_mlp, m->n_mlp, m->tcount);
    const int grow = cfg->loss_scale_growth_interval > 0 ? cfg->loss_scale_growth_interval : kGrowIntervalDefault;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, m->dacc, m->tcount, m->s, m->g_s, losses, B,
                       prec != NIF_PREC_FP32 ? 1 : 0, grow, cfg->beta1, cfg->beta2, cfg->fixed_task_weights);
    AdamParams A;
    A.tables = m->tables; A.g_tables = m->g_tables; A.m_tables = m->m_tables; A.v_tables = m->v_tables;
    A.tables_h = m->desc.table_dtype == NIF_TABLE_F16 ? m->tables_h : nullptr;
    A.mlp = m->mlp; A.g_mlp = m->g_mlp; A.m_mlp = m->m_mlp; A.v_mlp = m->v_mlp;
    A.s = m->s; A.g_s = m->g_s; A.m_s = m->m_s; A.v_s = m->v_s;
    A.n_table = m->n_table; A.n_mlp = m->n_mlp;
    A.lr_table = cfg->lr_table; A.lr_mlp = cfg->lr_mlp; A.lr_s = cfg->fixed_task_weights ? 0.f : cfg->lr_s;
    A.beta1 = cfg->beta1; A.beta2 = cfg->beta2; A.eps = cfg->eps;
    hipLaunchKernelGGL(k_adam, dim3(grid_for(m->n_table + m->n_mlp + 5)), dim3(256), 0, st, A, m->dacc, m->tcount);
    if ((rc = check_hip(hipGetLastError(), "train step launch"))) return rc;
    if ((rc = model_sync_mlp(m, st))) return rc;
    ++m->step;
    return NIF_OK;
}

}  // namespace nif
