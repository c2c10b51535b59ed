// Model parameters: FP32 masters in the canonical layouts, and the working copies the
// kernels read (FP16 tables; the MLP padded to a 16-row output layer in FP32, BF16 and FP16).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "nif_internal.hpp"
#include "nif_net.hpp"

namespace nif {

__global__ void k_sync_tables(const float* __restrict__ src, __half* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = __float2half_rn(src[i]);
}

struct LayerMap {
    int64_t w_off[kMaxLayers], b_off[kMaxLayers], wp_off[kMaxLayers], bp_off[kMaxLayers], wt_off[kMaxLayers];
    int32_t in[kMaxLayers], out[kMaxLayers], out_pad[kMaxLayers];
    int32_t n_layers;
};

// padded[i] <- canonical (rows beyond the real output count are zero)
__global__ void k_sync_mlp(LayerMap lm, const float* __restrict__ src, float* __restrict__ f32,
                           uint16_t* __restrict__ bf16, __half* __restrict__ f16) {
    const int layer = blockIdx.y;
    const int nin = lm.in[layer], nout = lm.out[layer], npad = lm.out_pad[layer];
    const int64_t nw = (int64_t)npad * nin;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw + npad; i += (int64_t)gridDim.x * blockDim.x) {
        float v;
        int64_t dst;
        if (i < nw) {
            const int64_t row = i / nin, col = i % nin;
            v = row < nout ? src[lm.w_off[layer] + row * nin + col] : 0.f;
            dst = lm.wp_off[layer] + i;
        } else {
            const int64_t row = i - nw;
            v = row < nout ? src[lm.b_off[layer] + row] : 0.f;
            dst = lm.bp_off[layer] + row;
        }
        f32[dst] = v;
        bf16[dst] = f2bf(v);
        f16[dst] = __float2half_rn(v);
        if (i < nw) {                   // transposed copy [in][out_pad] for the backward
            const int64_t row = i / nin, col = i % nin;
            const int64_t t = lm.wt_off[layer] + col * npad + row;
            f32[t] = v;
            bf16[t] = f2bf(v);
            f16[t] = __float2half_rn(v);
        }
    }
}

// First-layer weights in the order the fused kernels read them, so that each of a wave's
// weight loads is one contiguous block (8 or 4 whole cache lines) instead of 64 scattered rows.
// A level batch is LB levels (4 with two features per entry, 2 with three), whose LB Fd
// features fill t < LB Fd of a lane's 8 k-values.  Lane (q, j) of MFMA block ob, at the u-th
// PE combination of its quarter (c = qU + u) and level batch lb, reads
// W0[ob 16 + j][(c L + LB lb) Fd + t], t = 4h + k, as element k of half h; the padding
// (t >= LB Fd) and combinations past 2S are zero.
__global__ void k_sync_w0l(const float* __restrict__ w0, int E, int HW, int U, int L, int Fd, int n_comb,
                           float* __restrict__ f32, uint16_t* __restrict__ bf16, __half* __restrict__ f16, int64_t n) {
    const int LB = Fd == 2 ? 4 : 2;
    const int NLB = L / LB;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i;
        const int k = (int)(r & 3); r >>= 2;
        const int lane = (int)(r & 63); r >>= 6;
        const int h = (int)(r & 1); r >>= 1;
        const int lb = (int)(r % NLB); r /= NLB;
        const int u = (int)(r % U); r /= U;
        const int ob = (int)r;
        const int q = lane >> 4, j = lane & 15;
        const int c = q * U + u;
        const int t = 4 * h + k;
        const float v = c < n_comb && t < LB * Fd ? w0[(int64_t)(ob * 16 + j) * E + ((int64_t)c * L + LB * lb) * Fd + t] : 0.f;
        f32[i] = v;
        bf16[i] = f2bf(v);
        f16[i] = __float2half_rn(v);
    }
}

static int sync_w0l(nif_model* m, hipStream_t st) {
    const int L = m->desc.levels, HW = m->desc.hidden_width, n_comb = 2 * m->S, U = (n_comb + 3) >> 2;
    hipLaunchKernelGGL(k_sync_w0l, dim3(256), dim3(256), 0, st, m->mlp_pad_f32 + m->wp_off[0], m->E, HW, U, L,
                       m->desc.feat_dim, n_comb, m->w0l_f32, m->w0l_bf16, m->w0l_f16, m->n_w0l);
    return check_hip(hipGetLastError(), "k_sync_w0l");
}

static LayerMap layer_map(const nif_model* m) {
    LayerMap lm;
    memset(&lm, 0, sizeof(lm));
    lm.n_layers = m->n_layers;
    for (int i = 0; i < m->n_layers; ++i) {
        lm.w_off[i] = m->w_off[i]; lm.b_off[i] = m->b_off[i];
        lm.wp_off[i] = m->wp_off[i]; lm.bp_off[i] = m->bp_off[i]; lm.wt_off[i] = m->wt_off[i];
        lm.in[i] = m->dims[i]; lm.out[i] = m->dims[i + 1]; lm.out_pad[i] = m->dims_pad[i + 1];
    }
    return lm;
}

int model_sync_mlp(nif_model* m, hipStream_t st) {
    hipLaunchKernelGGL(k_sync_mlp, dim3(64, m->n_layers), dim3(256), 0, st, layer_map(m), m->mlp, m->mlp_pad_f32,
                       m->mlp_pad_bf16, m->mlp_pad_f16);
    const int rc = check_hip(hipGetLastError(), "k_sync_mlp");
    return rc ? rc : sync_w0l(m, st);
}

int model_sync_working(nif_model* m, hipStream_t st) {
    if (m->desc.table_dtype == NIF_TABLE_F16) {
        hipLaunchKernelGGL(k_sync_tables, dim3(2048), dim3(256), 0, st, m->tables, m->tables_h, m->n_table);
        int rc = check_hip(hipGetLastError(), "k_sync_tables");
        if (rc) return rc;
    }
    return model_sync_mlp(m, st);
}

template <typename T>
static int dalloc(T** p, int64_t n, const char* what) {
    if (hipMalloc((void**)p, sizeof(T) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(NIF_E_OOM, std::string("device allocation failed: ") + what);
    }
    return NIF_OK;
}

int model_alloc(nif_model* m) {
    const nif_model_desc& d = m->desc;
    m->S = d.concat_encoding ? 1 : 1 + 2 * d.pe_freqs;
    m->GW = d.concat_encoding ? 3 * (1 + 2 * d.pe_freqs) : 0;
    m->E = 2 * (m->S * d.levels * d.feat_dim + m->GW);
    m->H = 8 + d.n_materials;
    m->n_table = (int64_t)(d.per_sample_tables ? m->S : 1) * d.levels * ((int64_t)1 << d.log2_table) * d.feat_dim;
    m->dims.clear();
    m->dims.push_back(m->E);
    for (int i = 0; i < d.hidden_layers; ++i) m->dims.push_back(d.hidden_width);
    m->dims.push_back(m->H);
    m->n_layers = (int32_t)m->dims.size() - 1;
    m->dims_pad = m->dims;
    m->dims_pad.back() = 16;
    m->w_off.assign(m->n_layers, 0); m->b_off.assign(m->n_layers, 0);
    m->wp_off.assign(m->n_layers, 0); m->bp_off.assign(m->n_layers, 0); m->wt_off.assign(m->n_layers, 0);
    int64_t off = 0, offp = 0;
    for (int i = 0; i < m->n_layers; ++i) {
        m->w_off[i] = off; off += (int64_t)m->dims[i + 1] * m->dims[i];
        m->b_off[i] = off; off += m->dims[i + 1];
        m->wp_off[i] = offp; offp += (int64_t)m->dims_pad[i + 1] * m->dims_pad[i];
        m->bp_off[i] = offp; offp += m->dims_pad[i + 1];
    }
    for (int i = 0; i < m->n_layers; ++i) {
        m->wt_off[i] = offp; offp += (int64_t)m->dims_pad[i + 1] * m->dims_pad[i];
    }
    m->n_mlp = off;
    m->n_mlp_pad = offp;
    m->n_w0l = (int64_t)(d.hidden_width / 16) * ((2 * m->S + 3) / 4) * (d.levels / (d.feat_dim == 2 ? 4 : 2)) * 2 * 64 * 4;
    int rc;
    if ((rc = dalloc(&m->tables, m->n_table, "tables"))) return rc;
    if (d.table_dtype == NIF_TABLE_F16 && (rc = dalloc(&m->tables_h, m->n_table, "fp16 tables"))) return rc;
    if ((rc = dalloc(&m->mlp, m->n_mlp, "mlp"))) return rc;
    if ((rc = dalloc(&m->mlp_pad_f32, m->n_mlp_pad, "mlp f32"))) return rc;
    if ((rc = dalloc(&m->mlp_pad_bf16, m->n_mlp_pad, "mlp bf16"))) return rc;
    if ((rc = dalloc(&m->mlp_pad_f16, m->n_mlp_pad, "mlp f16"))) return rc;
    if ((rc = dalloc(&m->w0l_f32, m->n_w0l, "first layer f32"))) return rc;
    if ((rc = dalloc(&m->w0l_bf16, m->n_w0l, "first layer bf16"))) return rc;
    if ((rc = dalloc(&m->w0l_f16, m->n_w0l, "first layer f16"))) return rc;
    if ((rc = dalloc(&m->s, 8, "s"))) return rc;
    if ((rc = dalloc(&m->g_tables, m->n_table, "table grads"))) return rc;
    if ((rc = dalloc(&m->g_mlp, m->n_mlp, "mlp grads"))) return rc;
    if ((rc = dalloc(&m->g_s, 8, "s grads"))) return rc;
    if ((rc = dalloc(&m->m_tables, m->n_table, "adam m"))) return rc;
    if ((rc = dalloc(&m->v_tables, m->n_table, "adam v"))) return rc;
    if ((rc = dalloc(&m->m_mlp, m->n_mlp, "adam m"))) return rc;
    if ((rc = dalloc(&m->v_mlp, m->n_mlp, "adam v"))) return rc;
    if ((rc = dalloc(&m->m_s, 8, "adam m"))) return rc;
    if ((rc = dalloc(&m->v_s, 8, "adam v"))) return rc;
    if ((rc = dalloc(&m->counters, 8, "counters"))) return rc;
    if ((rc = dalloc(&m->dacc, 16, "train accumulators"))) return rc;
    if ((rc = dalloc(&m->tcount, 16, "train counters"))) return rc;
    // side stream of the backward (default priority) and its fork / join events
    if (hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return fail(NIF_E_DEVICE, "stream / event creation failed");
    }
    return NIF_OK;
}

void model_free(nif_model* m) {
    if (m->side) (void)hipStreamSynchronize(m->side);     // the backward's side work reads these buffers
    void* ps[] = {m->tables, m->tables_h, m->mlp, m->mlp_pad_f32, m->mlp_pad_bf16, m->mlp_pad_f16, m->s,
                  m->g_tables, m->g_mlp, m->g_s, m->m_tables, m->v_tables, m->m_mlp, m->v_mlp,
                  m->m_s, m->v_s, m->counters, m->dacc, m->tcount, m->zbuf, m->dz, m->acts, m->delta,
                  m->enc, m->enc_all, m->bwd_cnt, m->bwd_scan, m->bwd_val, m->w0l_f32, m->w0l_bf16, m->w0l_f16,
                  m->dw_part, m->ord_u32, m->ord_f32, m->ord_temp};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    if (m->ev_join) (void)hipEventDestroy(m->ev_join);
    if (m->side) (void)hipStreamDestroy(m->side);
}

}  // namespace nif
