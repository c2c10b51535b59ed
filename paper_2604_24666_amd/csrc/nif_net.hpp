// Hybrid encoding psi = phi(gamma(x)) and the intersection MLP, for one wavefront.
//
// Eq. (1) and "Combining Positional Encoding with the Grid Encoding": each rest-space point
// x (clamped to the unit cube) is expanded into S = 1 + 2F positional-encoding samples
// [x, (sin 2^k x + 1)/2, (cos 2^k x + 1)/2]; every sample is looked up in the same
// L-level grid (dense indexing where (N_l + 1)^3 fits the table, the Instant-NGP spatial
// hash otherwise) with trilinear interpolation; the features of the entry and exit points
// are concatenated (point, sample, level, feature) and fed to the MLP (Methodology: the
// network predicts hit, distance, normal, albedo and material).
//
// Precision.  The sin/cos samples and the grid position S * N_l are formed in FP64 (one FP32
// ulp of a sample moves a finest-level position by N_l / 2^24, which the interpolation turns
// into a relative feature error of ~1e-4); interpolation weights, features and the MLP run in
// FP32, or BF16/FP16 MFMA with FP32 accumulation.  sin/cos of 2^k x come from one FP64
// sincos and the double-angle recurrence.
//
// MLP on MFMA (v_mfma_f32_16x16x{4f32,16bf16_1k,16f16}).  The wave evaluates 16*CB
// segments at a time in transposed form: out^T[n_out x segs] = W[n_out x n_in] x in^T.
// Weights are the A operand (rows = output neurons), activations the B operand (columns =
// segments).  The 16x16 result tile of lane l holds neurons 4(l/16)+r, r < 4, of segment
// l%16, which is exactly the B-operand layout of the next layer's K-block, so hidden layers
// chain in registers.  For the first layer each lane computes the features the B operand
// needs: lane quarter q = l/16 evaluates levels [q L/4, (q+1) L/4) of segment l%16.
#pragma once
#include "nif_device.hpp"

namespace nif {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));

enum { P_FP32 = 0, P_BF16 = 1, P_FP16 = 2 };
constexpr int kMaxLayers = 10;
constexpr int kSegStride = 8;    // LDS floats per segment: x0 (3), pad, x1 (3), pad
constexpr int kZStride = 17;     // LDS floats per segment of head outputs (16 + pad)
#ifndef NIF_QUERY_CB
#define NIF_QUERY_CB 1
#endif
constexpr int kQueryCB = NIF_QUERY_CB;      // 16-segment column blocks per MLP pass in the fused query

struct EncParams {
    const void* tab;        // [sets][L][T][Fd] FP32 or FP16
    int32_t f16;
    int32_t L, log2T, F;
    int32_t Fd;             // features per entry: 2 or 3
    int32_t res[16];
    uint32_t dense_mask;    // bit l: level l indexed densely
    int64_t set_stride;     // entries per table set: L T with one set per PE sample, else 0
};

// First entry of the table set that PE sample s reads (the tables hold fewer than 2^32 entries).
__device__ __forceinline__ uint32_t set_offset(const EncParams& ep, int s) { return (uint32_t)s * (uint32_t)ep.set_stride; }
// Table set entry offset of PE combination c (point-major: c = p S + s).
__device__ __forceinline__ uint32_t combo_set_offset(const EncParams& ep, int c, int S) {
    return set_offset(ep, c >= S ? c - S : c);
}

struct NetParams {
    EncParams enc;
    const void* W[kMaxLayers];   // padded weights in the MLP precision, row-major [out][in]
    const void* W0L;             // the first layer again, in lane order (see k_sync_w0l)
    const float* b[kMaxLayers];  // padded FP32 biases
    int32_t n_hidden;            // hidden layers
    int32_t E;                   // encoding width (both points)
    int32_t H;                   // real head count
    int32_t dist_head;           // NIF_DIST_LOG_RELU or NIF_DIST_SIGMOID
    int32_t gamma_F;             // concatenated encoding: PE frequencies of the appended gamma (-1: none)
    int32_t E_phi;               // encoding columns of the grid part (the gamma part follows)
};

__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int PREC>
__device__ __forceinline__ shortx4 pack4(float a, float b, float c, float d) {
    shortx4 r;
    if constexpr (PREC == P_BF16) {
        r[0] = (short)f2bf(a); r[1] = (short)f2bf(b); r[2] = (short)f2bf(c); r[3] = (short)f2bf(d);
    } else {
        _Float16 h0 = (_Float16)a, h1 = (_Float16)b, h2 = (_Float16)c, h3 = (_Float16)d;
        r[0] = __builtin_bit_cast(short, h0); r[1] = __builtin_bit_cast(short, h1);
        r[2] = __builtin_bit_cast(short, h2); r[3] = __builtin_bit_cast(short, h3);
    }
    return r;
}

template <int PREC>
__device__ __forceinline__ floatx4 mfma16(shortx4 a, shortx4 b, floatx4 c) {
    if constexpr (PREC == P_BF16) return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(halfx4, a), __builtin_bit_cast(halfx4, b), c, 0, 0, 0);
}

__device__ __forceinline__ floatx4 mfma32(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Grid cell and FP32 weights of one sample coordinate at resolution N.
__device__ __forceinline__ void grid_axis(double s, int N, uint32_t& i0, float& w) {
    double pos = s * (double)N;
    double f = floor(pos);
    f = fmin(fmax(f, 0.0), (double)(N - 1));   // samples can leave [0, 1] by an ulp
    i0 = (uint32_t)f;
    w = (float)(pos - f);
}

__device__ __forceinline__ uint32_t grid_index(uint32_t vx, uint32_t vy, uint32_t vz, uint32_t n1, bool dense,
                                               uint32_t mask) {
    uint32_t hd = vx + n1 * (vy + n1 * vz);
    uint32_t hh = (vx ^ (vy * 2654435761u) ^ (vz * 805459861u)) & mask;
    return dense ? hd : hh;
}

// Trilinearly interpolated features of level l at one sample (any Fd; one load per feature):
// out[f], f < Fd.  The plain form, for the encoding on its own.
template <bool F16>
__device__ __forceinline__ void grid_lookup_any(const EncParams& ep, int l, double sx, double sy, double sz,
                                                uint32_t set_off, float* out) {
    const uint32_t mask = (1u << ep.log2T) - 1u;
    const int N = ep.res[l];
    const bool dense = (ep.dense_mask >> l) & 1u;
    const uint32_t n1 = (uint32_t)N + 1u;
    uint32_t ix, iy, iz;
    float wx, wy, wz;
    grid_axis(sx, N, ix, wx);
    grid_axis(sy, N, iy, wy);
    grid_axis(sz, N, iz, wz);
    const size_t base = (size_t)(set_off + ((uint32_t)l << ep.log2T));
    for (int f = 0; f < ep.Fd; ++f) out[f] = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const size_t e = (base + grid_index(ix + (c & 1), iy + ((c >> 1) & 1), iz + ((c >> 2) & 1), n1, dense, mask)) *
                         (size_t)ep.Fd;
        const float wt = ((c & 1) ? wx : 1.f - wx) * (((c >> 1) & 1) ? wy : 1.f - wy) * (((c >> 2) & 1) ? wz : 1.f - wz);
        for (int f = 0; f < ep.Fd; ++f) {
            const float v = F16 ? __half2float(reinterpret_cast<const __half*>(ep.tab)[e + f])
                                : reinterpret_cast<const float*>(ep.tab)[e + f];
            out[f] = fmaf(wt, v, out[f]);
        }
    }
}

// ------------------------------------------------------------------ wave-uniform level lookups
// The first layer of the fused network assigns lanes as (PE combination, segment): every
// lane of the wave looks up the same level at the same time, so the level's resolution,
// table offset and dense/hash choice are wave-uniform.  The two x-neighbouring corners of
// each (y, z) corner pair are fetched with one paired load: in a dense level they are
// adjacent entries; in a hashed level (x prime 1) the entries of x and x+1 are the two
// halves of one aligned pair when x is even, and a second single-entry load is issued
// only by lanes whose x is odd.

template <bool F16> struct TabTypes;
template <> struct TabTypes<true> { using E = uint32_t; using Pr = uint2; };   // half2 entries
template <> struct TabTypes<false> { using E = uint2; using Pr = uint4; };     // float2 entries

__device__ __forceinline__ float2 entry_f2(uint32_t e) {
    return __half22float2(__builtin_bit_cast(__half2, e));
}
__device__ __forceinline__ float2 entry_f2(uint2 e) {
    return make_float2(__uint_as_float(e.x), __uint_as_float(e.y));
}
__device__ __forceinline__ void pair_split(uint2 p, uint32_t& lo, uint32_t& hi) { lo = p.x; hi = p.y; }
__device__ __forceinline__ void pair_split(uint4 p, uint2& lo, uint2& hi) { lo = make_uint2(p.x, p.y); hi = make_uint2(p.z, p.w); }
__device__ __forceinline__ uint32_t sel(bool c, uint32_t a, uint32_t b) { return c ? a : b; }
__device__ __forceinline__ uint2 sel(bool c, uint2 a, uint2 b) { return make_uint2(c ? a.x : b.x, c ? a.y : b.y); }

// Sample positions of increasing PE combinations of one segment: the first sample of each
// point and frequency run comes from one FP64 sincos, the next frequency by the double-angle
// recurrence (sin 2a = 2 sin a cos a, cos 2a = (cos a - sin a)(cos a + sin a)).
struct PEWalk {
    double sn[3], cs[3];
    int p, k;                  // point and frequency index held in sn / cs (k < 0: none)
};

__device__ __forceinline__ void pe_walk(const float* sp, int c, int S, PEWalk& w, double out[3]) {
    const int p = c >= S ? 1 : 0;
    const int s = c - p * S;
    double x[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = fmin(fmax((double)sp[4 * p + a], 0.0), 1.0);
    if (s == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) out[a] = x[a];
        return;
    }
    const int k = (s - 1) >> 1;
    if (w.p == p && w.k >= 0 && k == w.k + 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double s1 = w.sn[a], c1 = w.cs[a];
            w.sn[a] = 2.0 * s1 * c1;
            w.cs[a] = (c1 - s1) * (c1 + s1);
        }
        w.k = k;
    } else if (!(w.p == p && w.k == k)) {
#pragma unroll
        for (int a = 0; a < 3; ++a) sincos(ldexp(x[a], k), &w.sn[a], &w.cs[a]);
        w.p = p;
        w.k = k;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = 0.5 * (((s & 1) ? w.sn[a] : w.cs[a]) + 1.0);
}

// Positional-encoding state of one point coordinate triple across the samples.
struct PEState {
    double x[3], sn[3], cs[3];
};

__device__ __forceinline__ void pe_begin(PEState& st, float x, float y, float z) {
    st.x[0] = fmin(fmax((double)x, 0.0), 1.0);
    st.x[1] = fmin(fmax((double)y, 0.0), 1.0);
    st.x[2] = fmin(fmax((double)z, 0.0), 1.0);
}

// Sample s (0..2F) of the point; must be called with s increasing from 0.
__device__ __forceinline__ void pe_sample(PEState& st, int s, double out[3]) {
    if (s == 0) {
        out[0] = st.x[0]; out[1] = st.x[1]; out[2] = st.x[2];
        return;
    }
    const int k = (s - 1) >> 1;
    if ((s & 1) == 1) {             // sin sample of frequency 2^k: advance the recurrence
        if (k == 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) sincos(st.x[a], &st.sn[a], &st.cs[a]);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double s1 = st.sn[a], c1 = st.cs[a];
                st.sn[a] = 2.0 * s1 * c1;
                st.cs[a] = (c1 - s1) * (c1 + s1);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) out[a] = 0.5 * (st.sn[a] + 1.0);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) out[a] = 0.5 * (st.cs[a] + 1.0);
    }
}

// ------------------------------------------------------------------ fixed-point sample positions
// A sample position v in [0, 1] as a 32-bit fixed-point fraction: f = round(v 2^32), capped
// at 2^32 - 1.  At resolution N the cell is floor(f N / 2^32) <= N - 1 and the weight the
// remaining fraction; against FP64 v N the position differs by at most N 2^-33 (2.4e-7 of a
// cell at N = 2048), far below the FP32 feature error.
__device__ __forceinline__ uint32_t to_fix32(double v) {
    const double t = fmin(fmax(v, 0.0), 1.0) * 4294967296.0 + 0.5;
    return t >= 4294967295.0 ? 0xffffffffu : (uint32_t)t;
}

__device__ __forceinline__ void fix_axis(uint32_t f, uint32_t N, uint32_t& i0, float& w) {
    const uint64_t pos = (uint64_t)f * N;
    i0 = (uint32_t)(pos >> 32);
    w = (float)(uint32_t)pos * 2.3283064365386963e-10f;   // 2^-32
}

// Interpolated features of levels l0 .. l0+LB-1 (wave-uniform) at one fixed-point sample
// position: feat[2k + f] = feature f of level l0 + k.
template <int LB, bool F16>
__device__ __forceinline__ void lookup_levels(const EncParams& ep, int l0, const uint32_t f[3], float feat[2 * LB],
                                              uint32_t set_off = 0) {
    using E = typename TabTypes<F16>::E;
    using Pr = typename TabTypes<F16>::Pr;
    const E* tab = reinterpret_cast<const E*>(ep.tab);
    const uint32_t mask = (1u << ep.log2T) - 1u;
    Pr A[LB][4];
    E B[LB][4];
    uint32_t swp[LB];
    uint32_t ixs[LB];
    float wx[LB], wy[LB], wz[LB];
#pragma unroll
    for (int k = 0; k < LB; ++k) {
        const int l = l0 + k;
        const uint32_t N = (uint32_t)ep.res[l];
        uint32_t ix, iy, iz;
        fix_axis(f[0], N, ix, wx[k]);
        fix_axis(f[1], N, iy, wy[k]);
        fix_axis(f[2], N, iz, wz[k]);
        ixs[k] = ix;
        swp[k] = 0u;
        const E* tl = tab + (set_off + ((uint32_t)l << ep.log2T));
        if ((ep.dense_mask >> l) & 1u) {
            const uint32_t n1 = N + 1u;
#pragma unroll
            for (int pp = 0; pp < 4; ++pp) {
                const uint32_t e = ix + n1 * ((iy + (pp & 1)) + n1 * (iz + (pp >> 1)));
                __builtin_memcpy(&A[k][pp], tl + e, sizeof(Pr));
            }
        } else {
#pragma unroll
            for (int pp = 0; pp < 4; ++pp) {
                const uint32_t hyz = ((iy + (pp & 1)) * 2654435761u) ^ ((iz + (pp >> 1)) * 805459861u);
                const uint32_t h0 = (ix ^ hyz) & mask;
                swp[k] |= (h0 & 1u) << pp;
                __builtin_memcpy(&A[k][pp], tl + (h0 & ~1u), sizeof(Pr));
            }
            if (ix & 1u) {
#pragma unroll
                for (int pp = 0; pp < 4; ++pp) {
                    const uint32_t hyz = ((iy + (pp & 1)) * 2654435761u) ^ ((iz + (pp >> 1)) * 805459861u);
                    B[k][pp] = tl[((ix + 1u) ^ hyz) & mask];
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < LB; ++k) {
        const bool dense = (ep.dense_mask >> (l0 + k)) & 1u;
        const bool odd = !dense && (ixs[k] & 1u);
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int pp = 0; pp < 4; ++pp) {
            E lo, hi;
            pair_split(A[k][pp], lo, hi);
            const bool swap = (swp[k] >> pp) & 1u;
            const E e0 = sel(swap, hi, lo);
            const E e1 = odd ? B[k][pp] : sel(swap, lo, hi);
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const int c = 2 * pp + cx;
                const float wt = (cx ? wx[k] : 1.f - wx[k]) * (((c >> 1) & 1) ? wy[k] : 1.f - wy[k]) *
                                 (((c >> 2) & 1) ? wz[k] : 1.f - wz[k]);
                const float2 v = entry_f2(cx ? e1 : e0);
                acc.x = fmaf(wt, v.x, acc.x);
                acc.y = fmaf(wt, v.y, acc.y);
            }
        }
        feat[2 * k] = acc.x;
        feat[2 * k + 1] = acc.y;
    }
}

// Three-feature entries (12 or 6 bytes, no aligned pairs): every corner is its own load, all
// 8 LB of them issued before any is used.  feat[3k + f] = feature f of level l0 + k.
template <int LB, bool F16>
__device__ __forceinline__ void lookup_levels3(const EncParams& ep, int l0, const uint32_t f[3], float feat[3 * LB],
                                               uint32_t set_off = 0) {
    const uint32_t mask = (1u << ep.log2T) - 1u;
    uint32_t idx[LB][8];
    float wx[LB], wy[LB], wz[LB];
#pragma unroll
    for (int k = 0; k < LB; ++k) {
        const int l = l0 + k;
        const uint32_t N = (uint32_t)ep.res[l];
        uint32_t ix, iy, iz;
        fix_axis(f[0], N, ix, wx[k]);
        fix_axis(f[1], N, iy, wy[k]);
        fix_axis(f[2], N, iz, wz[k]);
        const bool dense = (ep.dense_mask >> l) & 1u;
        const uint32_t base = set_off + ((uint32_t)l << ep.log2T);
#pragma unroll
        for (int c = 0; c < 8; ++c)
            idx[k][c] = base + grid_index(ix + (c & 1), iy + ((c >> 1) & 1), iz + ((c >> 2) & 1), N + 1u, dense, mask);
    }
    float v[LB][8][3];
#pragma unroll
    for (int k = 0; k < LB; ++k)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const size_t e = (size_t)idx[k][c] * 3;
            if constexpr (F16) {
                const __half* t = reinterpret_cast<const __half*>(ep.tab) + e;
                v[k][c][0] = __half2float(t[0]); v[k][c][1] = __half2float(t[1]); v[k][c][2] = __half2float(t[2]);
            } else {
                const float* t = reinterpret_cast<const float*>(ep.tab) + e;
                v[k][c][0] = t[0]; v[k][c][1] = t[1]; v[k][c][2] = t[2];
            }
        }
#pragma unroll
    for (int k = 0; k < LB; ++k) {
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float wt = ((c & 1) ? wx[k] : 1.f - wx[k]) * (((c >> 1) & 1) ? wy[k] : 1.f - wy[k]) *
                             (((c >> 2) & 1) ? wz[k] : 1.f - wz[k]);
            a0 = fmaf(wt, v[k][c][0], a0);
            a1 = fmaf(wt, v[k][c][1], a1);
            a2 = fmaf(wt, v[k][c][2], a2);
        }
        feat[3 * k] = a0;
        feat[3 * k + 1] = a1;
        feat[3 * k + 2] = a2;
    }
}

// ------------------------------------------------------------------ one MLP pass
// The wave evaluates segments [seg_base, seg_base + 16*CB) whose rest-space points sit in
// s_seg (kSegStride floats each).  acc[ob][cb] holds the 16x16 MFMA tile of output rows
// [16 ob, 16 ob + 16) of column block cb: lane (q, j) has rows 16 ob + 4q + r of segment
// seg_base + 16 cb + j.

template <int HW, int CB>
__device__ __forceinline__ void layer1_bias(const NetParams& np, floatx4 (&acc)[HW / 16][CB]) {
    const int q = lane_id() >> 4;
#pragma unroll
    for (int ob = 0; ob < HW / 16; ++ob) {
        const float4 bb = *reinterpret_cast<const float4*>(np.b[0] + ob * 16 + 4 * q);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[ob][cb] = floatx4{bb.x, bb.y, bb.z, bb.w};
    }
}

// Layer 1 restricted to levels [lb, le) (a multiple of LB each), added to acc.  Lane (q, j)
// takes the PE combinations c = qU .. qU + U - 1 (point-major, 2S in all, U = ceil(2S / 4))
// of segment j in order, so its samples follow the double-angle recurrence; the wave walks
// the levels in batches of LB, all lanes on the same level.  A batch gives each lane 8 MFMA
// k-values: the LB FD features of (its combination, level batch) in encoding order, zero-padded
// (FD = 2: 4 levels, 8 features; FD = 3: 2 levels, 6 features and 2 zeros); the lane loads the
// matching lane-ordered weights (zero at the padding).
// enc_out (nullable): the features are also stored to enc_out[seg_g0 + seg][E].
template <int HW, int CB, int PREC, int FD>
__device__ __forceinline__ void layer1_levels(const NetParams& np, const float* s_seg, int seg_base, int lb, int le,
                                              floatx4 (&acc)[HW / 16][CB], float* enc_out, int64_t seg_g0,
                                              int64_t n_valid) {
    static_assert(FD == 2 || FD == 3, "2 or 3 features per entry");
    constexpr int LB = FD == 2 ? 4 : 2;      // levels per batch
    constexpr int NR = LB * FD;              // real features per lane per batch
    constexpr int NF = 8;                    // MFMA k-values per lane per batch
    constexpr int OB = HW / 16;
    const int lane = lane_id();
    const int q = lane >> 4, j = lane & 15;
    const int L = np.enc.L;
    const int S = 1 + 2 * np.enc.F;
    const int E = np.E;
    const int n_comb = 2 * S;
    const int U = (n_comb + 3) >> 2;           // combinations per lane quarter: q U .. q U + U - 1
    PEWalk pw[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) { pw[cb].p = -1; pw[cb].k = -1; }
    for (int u = 0; u < U; ++u) {
        const int c_raw = q * U + u;
        const bool live = c_raw < n_comb;
        const int c = live ? c_raw : 0;
        const uint32_t soff = combo_set_offset(np.enc, c, S);
        uint32_t smp[CB][3];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            smp[cb][0] = smp[cb][1] = smp[cb][2] = 0x80000000u;
            if (live) {
                double v[3];
                pe_walk(s_seg + (seg_base + cb * 16 + j) * kSegStride, c, S, pw[cb], v);
#pragma unroll
                for (int a = 0; a < 3; ++a) smp[cb][a] = to_fix32(v[a]);
            }
        }
        for (int l0 = lb; l0 < le; l0 += LB) {
            float feat[CB][NF];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                if constexpr (FD == 2) {
                    if (np.enc.f16) {
                        lookup_levels<LB, true>(np.enc, l0, smp[cb], feat[cb], soff);
                    } else {     // FP32 entries are twice the size: two levels at a time
#pragma unroll
                        for (int h = 0; h < LB; h += 2) lookup_levels<2, false>(np.enc, l0 + h, smp[cb], feat[cb] + 2 * h, soff);
                    }
                } else {
                    if (np.enc.f16) lookup_levels3<LB, true>(np.enc, l0, smp[cb], feat[cb], soff);
                    else lookup_levels3<LB, false>(np.enc, l0, smp[cb], feat[cb], soff);
#pragma unroll
                    for (int t = NR; t < NF; ++t) feat[cb][t] = 0.f;
                }
                if (!live) {
#pragma unroll
                    for (int t = 0; t < NF; ++t) feat[cb][t] = 0.f;
                }
            }
            const int e0 = (c * L + l0) * FD;
            if (enc_out) {
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int64_t seg = seg_g0 + cb * 16 + j;
                    if (live && seg < n_valid) {
                        if constexpr (FD == 2) {
                            float4* dst = reinterpret_cast<float4*>(enc_out + seg * E + e0);
#pragma unroll
                            for (int h = 0; h < NF / 4; ++h)
                                dst[h] = make_float4(feat[cb][4 * h], feat[cb][4 * h + 1], feat[cb][4 * h + 2], feat[cb][4 * h + 3]);
                        } else {
#pragma unroll
                            for (int t = 0; t < NR; ++t) enc_out[seg * E + e0 + t] = feat[cb][t];
                        }
                    }
                }
            }
#pragma unroll
            for (int ob = 0; ob < OB; ++ob) {
                // lane-ordered weights: half h of this lane's 8 at wl + (h 64 + lane) 4
                const size_t wl = (((size_t)ob * U + u) * (L / LB) + l0 / LB) * 512;
                if constexpr (PREC == P_FP32) {
                    const float* w = reinterpret_cast<const float*>(np.W0L) + wl + lane * 4;
                    float wf[NF];
#pragma unroll
                    for (int h = 0; h < NF / 4; ++h) {
                        const float4 wv = *reinterpret_cast<const float4*>(w + h * 256);
                        wf[4 * h] = wv.x; wf[4 * h + 1] = wv.y; wf[4 * h + 2] = wv.z; wf[4 * h + 3] = wv.w;
                    }
#pragma unroll
                    for (int t = 0; t < NR; ++t)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) acc[ob][cb] = mfma32(wf[t], feat[cb][t], acc[ob][cb]);
                } else {
                    const uint16_t* w = reinterpret_cast<const uint16_t*>(np.W0L) + wl + lane * 4;
#pragma unroll
                    for (int t = 0; t < NF / 4; ++t) {
                        const shortx4 wa = *reinterpret_cast<const shortx4*>(w + t * 256);
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) {
                            const shortx4 fb = pack4<PREC>(feat[cb][4 * t], feat[cb][4 * t + 1], feat[cb][4 * t + 2],
                                                           feat[cb][4 * t + 3]);
                            acc[ob][cb] = mfma16<PREC>(wa, fb, acc[ob][cb]);
                        }
                    }
                }
            }
        }
    }
}

// ReLU of the first layer's pre-activations in acc, the hidden layers and the output layer;
// writes the 16 padded head outputs to s_z.  acts (nullable): hidden activations are also
// stored to acts[layer][seg_g0 + seg][HW].
template <int HW, int CB, int PREC>
__device__ __forceinline__ void mlp_tail(const NetParams& np, floatx4 (&acc)[HW / 16][CB], int seg_base, float* s_z,
                                         float* acts, int64_t act_stride_layer, int64_t seg_g0, int64_t n_valid) {
    constexpr int OB = HW / 16;
    const int lane = lane_id();
    const int q = lane >> 4, j = lane & 15;
    // ---- hidden layers 2..n_hidden, output layer
    for (int layer = 1; layer <= np.n_hidden; ++layer) {
        // ReLU of the previous layer's outputs (and optional store)
#pragma unroll
        for (int ob = 0; ob < OB; ++ob)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[ob][cb][r] = fmaxf(acc[ob][cb][r], 0.f);
                if (acts) {
                    const int64_t seg = seg_g0 + cb * 16 + j;
                    if (seg < n_valid) {
                        float* dst = acts + (int64_t)(layer - 1) * act_stride_layer + seg * HW + ob * 16 + 4 * q;
                        *reinterpret_cast<float4*>(dst) = make_float4(acc[ob][cb][0], acc[ob][cb][1], acc[ob][cb][2], acc[ob][cb][3]);
                    }
                }
            }
        const bool is_out = layer == np.n_hidden;
        if (!is_out) {
            floatx4 nxt[OB][CB];
            const float* bl = np.b[layer];
#pragma unroll
            for (int ob = 0; ob < OB; ++ob) {
                const float4 bb = *reinterpret_cast<const float4*>(bl + ob * 16 + 4 * q);
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) nxt[ob][cb] = floatx4{bb.x, bb.y, bb.z, bb.w};
            }
            // the layer's input as B operands, converted once for all output blocks
            shortx4 hp[OB][CB];
            if constexpr (PREC != P_FP32) {
#pragma unroll
                for (int ob = 0; ob < OB; ++ob)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        hp[ob][cb] = pack4<PREC>(acc[ob][cb][0], acc[ob][cb][1], acc[ob][cb][2], acc[ob][cb][3]);
            }
#pragma unroll
            for (int oo = 0; oo < OB; ++oo)
#pragma unroll
                for (int ob = 0; ob < OB; ++ob) {
                    if constexpr (PREC == P_FP32) {
                        const float4 wv = *reinterpret_cast<const float4*>(
                            reinterpret_cast<const float*>(np.W[layer]) + (size_t)(oo * 16 + j) * HW + ob * 16 + 4 * q);
                        const float wf[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb) nxt[oo][cb] = mfma32(wf[r], acc[ob][cb][r], nxt[oo][cb]);
                    } else {
                        const shortx4 wa = *reinterpret_cast<const shortx4*>(
                            reinterpret_cast<const uint16_t*>(np.W[layer]) + (size_t)(oo * 16 + j) * HW + ob * 16 + 4 * q);
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) nxt[oo][cb] = mfma16<PREC>(wa, hp[ob][cb], nxt[oo][cb]);
                    }
                }
#pragma unroll
            for (int ob = 0; ob < OB; ++ob)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[ob][cb] = nxt[ob][cb];
        } else {
            floatx4 out[CB];
            const float4 bb = *reinterpret_cast<const float4*>(np.b[layer] + 4 * q);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) out[cb] = floatx4{bb.x, bb.y, bb.z, bb.w};
#pragma unroll
            for (int ob = 0; ob < OB; ++ob) {
                if constexpr (PREC == P_FP32) {
                    const float4 wv = *reinterpret_cast<const float4*>(
                        reinterpret_cast<const float*>(np.W[layer]) + (size_t)j * HW + ob * 16 + 4 * q);
                    const float wf[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) out[cb] = mfma32(wf[r], acc[ob][cb][r], out[cb]);
                } else {
                    const shortx4 wa = *reinterpret_cast<const shortx4*>(
                        reinterpret_cast<const uint16_t*>(np.W[layer]) + (size_t)j * HW + ob * 16 + 4 * q);
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        const shortx4 hb = pack4<PREC>(acc[ob][cb][0], acc[ob][cb][1], acc[ob][cb][2], acc[ob][cb][3]);
                        out[cb] = mfma16<PREC>(wa, hb, out[cb]);
                    }
                }
            }
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) s_z[(seg_base + cb * 16 + j) * kZStride + 4 * q + r] = out[cb][r];
        }
    }
}

// Raw gamma value v of a segment (concatenated encoding): point v / GW, then sample s and axis a
// of value 3 s + a: x, sin 2^k x or cos 2^k x of the clamped coordinate.
__device__ __forceinline__ float gamma_value(const float* seg, int v, int GW) {
    const int p = v >= GW ? 1 : 0, r = v - p * GW, s = r / 3, a = r - 3 * s;
    const float x = fminf(fmaxf(seg[4 * p + a], 0.f), 1.f);
    if (s == 0) return x;
    const float f = (float)(1 << ((s - 1) >> 1));
    return (s - 1) & 1 ? cosf(f * x) : sinf(f * x);
}

// First-layer contribution of the appended gamma values (columns E_phi .. E_phi + 2 GW) of
// segments [seg_base, seg_base + 16 CB): lane (q, j) supplies value k of segment j for the
// MFMA k-index it owns; enc_out (nullable) also receives the values.
template <int HW, int CB, int PREC>
__device__ __forceinline__ void layer1_gamma(const NetParams& np, const float* s_seg, int seg_base,
                                             floatx4 (&acc)[HW / 16][CB], float* enc_out, int64_t seg_g0,
                                             int64_t n_valid) {
    constexpr int OB = HW / 16;
    constexpr int KL = PREC == P_FP32 ? 1 : 4;    // k values per lane per MFMA
    const int lane = lane_id();
    const int q = lane >> 4, j = lane & 15;
    const int GW = 3 * (1 + 2 * np.gamma_F), NV = 2 * GW;
    for (int v0 = 0; v0 < NV; v0 += 4 * KL) {
        float g[CB][KL];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const float* my = s_seg + (seg_base + cb * 16 + j) * kSegStride;
#pragma unroll
            for (int i = 0; i < KL; ++i) {
                const int v = v0 + q * KL + i;
                g[cb][i] = v < NV ? gamma_value(my, v, GW) : 0.f;
            }
            if (enc_out) {
                const int64_t seg = seg_g0 + cb * 16 + j;
                if (seg < n_valid)
#pragma unroll
                    for (int i = 0; i < KL; ++i) {
                        const int v = v0 + q * KL + i;
                        if (v < NV) enc_out[seg * np.E + np.E_phi + v] = g[cb][i];
                    }
            }
        }
#pragma unroll
        for (int ob = 0; ob < OB; ++ob) {
            const size_t row = (size_t)(ob * 16 + j) * np.E + np.E_phi;
            if constexpr (PREC == P_FP32) {
                const int v = v0 + q;
                const float w = v < NV ? reinterpret_cast<const float*>(np.W[0])[row + v] : 0.f;
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[ob][cb] = mfma32(w, g[cb][0], acc[ob][cb]);
            } else {
                const uint16_t* wr = reinterpret_cast<const uint16_t*>(np.W[0]) + row;
                shortx4 wa;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int v = v0 + q * 4 + i;
                    wa[i] = v < NV ? (short)wr[v] : (short)0;
                }
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const shortx4 gb = pack4<PREC>(g[cb][0], g[cb][1], g[cb][2], g[cb][3]);
                    acc[ob][cb] = mfma16<PREC>(wa, gb, acc[ob][cb]);
                }
            }
        }
    }
}

// Whole network on segments [seg_base, seg_base + 16*CB); acts / enc_out as above.  GAMMA:
// the concatenated encoding, FD: features per table entry (each compiled separately, so the
// other kernels carry none of their code).
template <int HW, int CB, int PREC, bool GAMMA = false, int FD = 2>
__device__ __forceinline__ void net_pass(const NetParams& np, const float* s_seg, int seg_base, float* s_z,
                                         float* acts, int64_t act_stride_layer, int64_t seg_g0, int64_t n_valid,
                                         float* enc_out = nullptr) {
    floatx4 acc[HW / 16][CB];
    layer1_bias<HW, CB>(np, acc);
    layer1_levels<HW, CB, PREC, FD>(np, s_seg, seg_base, 0, np.enc.L, acc, enc_out, seg_g0, n_valid);
    if constexpr (GAMMA) layer1_gamma<HW, CB, PREC>(np, s_seg, seg_base, acc, enc_out, seg_g0, n_valid);
    mlp_tail<HW, CB, PREC>(np, acc, seg_base, s_z, acts, act_stride_layer, seg_g0, n_valid);
}

// Make this wave's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace nif
