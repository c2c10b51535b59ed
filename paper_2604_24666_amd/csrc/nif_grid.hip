// Rest-space voxelization and the per-pose deformed acceleration grid.
//
// Methodology: the geometry is voxelized once in rest space; every pose deforms the voxels,
// and rays are traced against the deformed voxels.  Because deformed voxels no longer have
// uniform extents, the voxel under a point cannot be found by index arithmetic ("Voxel
// Traversal under Deformation"); the paper finds the first voxel with a BVH.  Here each pose
// gets a uniform bin grid over its deformed bounding box instead: every occupied voxel is
// listed in the bins its (padded) deformed box overlaps, and a ray walks the bins with a
// 3D-DDA, testing the listed voxels exactly.  The bins only narrow the search; the set of
// voxels a ray crosses, and their order, come from the exact voxel tests.
//
// Build, per pose, all on the device:
//   1 lattice vertices V_ijk = D(i/N, j/N, k/N)              (float4, x fastest)
//   2 occupied voxels compacted once (shared by all poses)
//   3 padded deformed boxes of the occupied voxels, reduced to the pose's bounding box
//   4 bin sizes; per-bin reference counts; exclusive scan; fill.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "nif_internal.hpp"

namespace nif {

// ------------------------------------------------------------------ voxelization

__global__ void k_voxelize(int32_t kind, const float* __restrict__ sp, int32_t N,
                           uint8_t* __restrict__ occ) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)N * N * N;
    if (c >= n) return;
    int i = (int)(c % N), j = (int)((c / N) % N), k = (int)(c / ((int64_t)N * N));
    float lo = INFINITY, hi = -INFINITY;
    const float inv = 1.f / (float)N;
    for (int cz = 0; cz <= 4; ++cz)
        for (int cy = 0; cy <= 4; ++cy)
            for (int cx = 0; cx <= 4; ++cx) {
                float3 p = make_float3((i + 0.25f * cx) * inv, (j + 0.25f * cy) * inv, (k + 0.25f * cz) * inv);
                float v = scene_f(kind, sp, p);
                lo = fminf(lo, v);
                hi = fmaxf(hi, v);
            }
    occ[c] = (lo <= 0.f && hi >= 0.f) ? 1 : 0;
}

int voxelize_launch(int32_t kind, const float* sp, int32_t N, uint8_t* occ, hipStream_t st) {
    int64_t n = (int64_t)N * N * N;
    hipLaunchKernelGGL(k_voxelize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, kind, sp, N, occ);
    return check_hip(hipGetLastError(), "voxelize launch");
}

// ------------------------------------------------------------------ build kernels

__global__ void k_vertices(const PoseDev* __restrict__ poses, int32_t N, float4* __restrict__ V) {
    const int p = blockIdx.y;
    const PoseDev P = poses[p];
    int64_t nv = (int64_t)(N + 1) * (N + 1) * (N + 1);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    int i = (int)(v % (N + 1)), j = (int)((v / (N + 1)) % (N + 1)), k = (int)(v / ((int64_t)(N + 1) * (N + 1)));
    const float inv = 1.f / (float)N;
    float3 q = deform(P, make_float3(i * inv, j * inv, k * inv));
    V[P.vert_off + v] = make_float4(q.x, q.y, q.z, 0.f);
}

__global__ void k_compact(const uint8_t* __restrict__ occ, int64_t n, int32_t* __restrict__ list,
                          int32_t* __restrict__ count) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool o = c < n && occ[c];
    uint64_t m = __ballot(o);
    int base = 0;
    if (lane_id() == 0 && m) base = atomicAdd(count, popc64(m));
    base = __shfl(base, 0);
    if (o) list[base + rank_below(m)] = (int32_t)c;
}

// Order-preserving map of floats to signed ints (for atomic min/max of floats).
__device__ inline int32_t f2ord(float f) {
    int32_t i = __float_as_int(f);
    return i >= 0 ? i : (int32_t)(i ^ 0x7fffffff);
}
__host__ inline float ord2f_host(int32_t i) {
    int32_t r = i >= 0 ? i : (int32_t)(i ^ 0x7fffffff);
    float f;
    memcpy(&f, &r, 4);
    return f;
}

__device__ inline void cell_box(const float4* __restrict__ V, int32_t N, int32_t cell, float lo[3], float hi[3]) {
    int i = cell % N, j = (cell / N) % N, k = cell / (N * N);
    lo[0] = lo[1] = lo[2] = INFINITY;
    hi[0] = hi[1] = hi[2] = -INFINITY;
    for (int m = 0; m < 8; ++m) {
        int64_t vi = (int64_t)(i + (m & 1)) + (int64_t)(N + 1) * ((j + ((m >> 1) & 1)) + (int64_t)(N + 1) * (k + (m >> 2)));
        float4 v = V[vi];
        lo[0] = fminf(lo[0], v.x); lo[1] = fminf(lo[1], v.y); lo[2] = fminf(lo[2], v.z);
        hi[0] = fmaxf(hi[0], v.x); hi[1] = fmaxf(hi[1], v.y); hi[2] = fmaxf(hi[2], v.z);
    }
    for (int a = 0; a < 3; ++a) { lo[a] -= kBinPad; hi[a] += kBinPad; }
}

// bbox[p][6] as ordered ints: min x,y,z then max x,y,z
__global__ void k_pose_bbox(const PoseDev* __restrict__ poses, const float4* __restrict__ V, int32_t N,
                            const int32_t* __restrict__ list, int32_t n_occ, int32_t* __restrict__ bbox) {
    const int p = blockIdx.y;
    const float4* Vp = V + poses[p].vert_off;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_occ; t += (int64_t)gridDim.x * blockDim.x) {
        float a[3], b[3];
        cell_box(Vp, N, list[t], a, b);
        for (int c = 0; c < 3; ++c) { lo[c] = fminf(lo[c], a[c]); hi[c] = fmaxf(hi[c], b[c]); }
    }
    for (int c = 0; c < 3; ++c) {
        for (int off = 32; off > 0; off >>= 1) {
            lo[c] = fminf(lo[c], __shfl_xor(lo[c], off));
            hi[c] = fmaxf(hi[c], __shfl_xor(hi[c], off));
        }
    }
    if (lane_id() == 0) {
        for (int c = 0; c < 3; ++c) {
            atomicMin(&bbox[6 * p + c], f2ord(lo[c]));
            atomicMax(&bbox[6 * p + 3 + c], f2ord(hi[c]));
        }
    }
}

__device__ inline void box_bins(const PoseDev& P, const float lo[3], const float hi[3], int b0[3], int b1[3]) {
    for (int a = 0; a < 3; ++a) {
        int x0 = (int)floorf((lo[a] - P.lo[a]) * P.inv_bs[a]);
        int x1 = (int)floorf((hi[a] - P.lo[a]) * P.inv_bs[a]);
        b0[a] = min(max(x0, 0), P.nb[a] - 1);
        b1[a] = min(max(x1, 0), P.nb[a] - 1);
    }
}

__global__ void k_bin_count(const PoseDev* __restrict__ poses, const float4* __restrict__ V, int32_t N,
                            const int32_t* __restrict__ list, int32_t n_occ, int32_t* __restrict__ counts) {
    const int p = blockIdx.y;
    const PoseDev P = poses[p];
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_occ || P.empty) return;
    float lo[3], hi[3];
    cell_box(V + P.vert_off, N, list[t], lo, hi);
    int b0[3], b1[3];
    box_bins(P, lo, hi, b0, b1);
    int32_t* cnt = counts + P.bin_off;
    for (int z = b0[2]; z <= b1[2]; ++z)
        for (int y = b0[1]; y <= b1[1]; ++y)
            for (int x = b0[0]; x <= b1[0]; ++x)
                atomicAdd(&cnt[x + P.nb[0] * (y + P.nb[1] * z)], 1);
}

// Exclusive scan of counts[0..n) into start[0..n] by one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) k_scan(const PoseDev* __restrict__ poses, const int32_t* __restrict__ counts,
                                               int32_t* __restrict__ start, int32_t* __restrict__ totals) {
    const int p = blockIdx.x;
    const PoseDev P = poses[p];
    const int64_t n = (int64_t)P.nb[0] * P.nb[1] * P.nb[2];
    const int32_t* c = counts + P.bin_off;
    int32_t* s = start + P.bin_off;
    __shared__ int32_t part[1024];
    const int T = blockDim.x;
    const int64_t per = (n + T - 1) / T;
    const int64_t a = min(n, (int64_t)threadIdx.x * per), b = min(n, a + per);
    int32_t sum = 0;
    for (int64_t i = a; i < b; ++i) sum += c[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        int32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - sum;   // exclusive prefix of this thread's range
    for (int64_t i = a; i < b; ++i) { s[i] = run; run += c[i]; }
    if (threadIdx.x == T - 1) { s[n] = part[T - 1]; totals[p] = part[T - 1]; }
}

// Per-pose offsets into the shared reference list (one thread).  A pose whose references do
// not fit the allocated capacity is marked empty (its rays then miss) and flagged.
__global__ void k_ref_offsets(PoseDev* __restrict__ poses, int n_poses, const int32_t* __restrict__ totals,
                              int64_t capacity, int32_t* __restrict__ overflow) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t off = 0;
    int32_t ov = 0;
    for (int p = 0; p < n_poses; ++p) {
        poses[p].ref_off = off;
        if (off + totals[p] > capacity) { poses[p].empty = 1; ov = 1; }
        else off += totals[p];
    }
    *overflow = ov;
}

// Bin-grid origin and bin size of every pose from its bounding box (bins per axis fixed).
__global__ void k_pose_bins(PoseDev* __restrict__ poses, int n_poses, const int32_t* __restrict__ bbox, int32_t n_occ) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_poses) return;
    PoseDev& q = poses[p];
    q.empty = n_occ == 0;
    for (int c = 0; c < 3; ++c) {
        const int32_t ilo = bbox[6 * p + c], ihi = bbox[6 * p + 3 + c];
        float lo = __int_as_float(ilo >= 0 ? ilo : (ilo ^ 0x7fffffff));
        float hi = __int_as_float(ihi >= 0 ? ihi : (ihi ^ 0x7fffffff));
        if (q.empty) { lo = 0.f; hi = 1.f; }
        q.lo[c] = lo;
        q.bs[c] = fmaxf((hi - lo) / q.nb[c], 1e-6f);
        q.inv_bs[c] = 1.f / q.bs[c];
    }
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

__global__ void k_bbox_init(int32_t* __restrict__ bbox, int n_poses) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * n_poses) return;
    bbox[i] = (i % 6) < 3 ? 0x7f800000 : (int32_t)(0xff800000u ^ 0x7fffffffu);
}

__global__ void k_bin_fill(const PoseDev* __restrict__ poses, const float4* __restrict__ V, int32_t N,
                           const int32_t* __restrict__ list, int32_t n_occ, const int32_t* __restrict__ start,
                           int32_t* __restrict__ cursor, int32_t* __restrict__ cells) {
    const int p = blockIdx.y;
    const PoseDev P = poses[p];
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_occ || P.empty) return;
    const int32_t cell = list[t];
    float lo[3], hi[3];
    cell_box(V + P.vert_off, N, cell, lo, hi);
    int b0[3], b1[3];
    box_bins(P, lo, hi, b0, b1);
    const int32_t* st = start + P.bin_off;
    int32_t* cur = cursor + P.bin_off;
    int32_t* out = cells + P.ref_off;
    for (int z = b0[2]; z <= b1[2]; ++z)
        for (int y = b0[1]; y <= b1[1]; ++y)
            for (int x = b0[0]; x <= b1[0]; ++x) {
                int b = x + P.nb[0] * (y + P.nb[1] * z);
                out[st[b] + atomicAdd(&cur[b], 1)] = cell;
            }
}

// Sort each bin's list by voxel id (insertion sort; lists are short) so the build is
// deterministic.
__global__ void k_bin_sort(const PoseDev* __restrict__ poses, const int32_t* __restrict__ start,
                           int32_t* __restrict__ cells) {
    const int p = blockIdx.y;
    const PoseDev P = poses[p];
    int64_t nb = (int64_t)P.nb[0] * P.nb[1] * P.nb[2];
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb || P.empty) return;
    const int32_t* st = start + P.bin_off;
    int32_t* c = cells + P.ref_off;
    for (int32_t i = st[b] + 1; i < st[b + 1]; ++i) {
        int32_t v = c[i], j = i - 1;
        while (j >= st[b] && c[j] > v) { c[j + 1] = c[j]; --j; }
        c[j + 1] = v;
    }
}

// ------------------------------------------------------------------ host orchestration

void grid_free(nif_grid* g) {
    void* ps[] = {g->poses, g->verts, g->bin_start, g->bin_cells, g->list, g->counts, g->scratch, g->order_pre};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    g->poses = nullptr; g->verts = nullptr; g->bin_start = nullptr; g->bin_cells = nullptr;
    g->list = nullptr; g->counts = nullptr; g->scratch = nullptr; g->order_pre = nullptr;
}

// scratch layout: bbox [6 P] | totals [P] | overflow [1] | n_occ [1]
static int32_t* sc_bbox(nif_grid* g) { return g->scratch; }
static int32_t* sc_totals(nif_grid* g) { return g->scratch + 6 * g->n_poses; }
static int32_t* sc_overflow(nif_grid* g) { return g->scratch + 7 * g->n_poses; }
static int32_t* sc_nocc(nif_grid* g) { return g->scratch + 7 * g->n_poses + 1; }

// Vertices, boxes, bin sizes, counts, scan and per-pose offsets; fills the reference lists
// when `fill`.  Device work only: no allocation, no synchronisation.
static int grid_rebin(nif_grid* g, bool fill, hipStream_t st) {
    const int P = g->n_poses, N = g->N;
    const int64_t nv = (int64_t)(N + 1) * (N + 1) * (N + 1);
    const int32_t n_occ = (int32_t)g->n_occupied;
    hipLaunchKernelGGL(k_vertices, dim3((unsigned)((nv + 255) / 256), P), dim3(256), 0, st, g->poses, N, g->verts);
    hipLaunchKernelGGL(k_bbox_init, dim3((6 * P + 255) / 256), dim3(256), 0, st, sc_bbox(g), P);
    if (n_occ > 0) {
        unsigned nblk = (unsigned)std::min<int64_t>((n_occ + 255) / 256, 1024);
        hipLaunchKernelGGL(k_pose_bbox, dim3(nblk, P), dim3(256), 0, st, g->poses, g->verts, N, g->list, n_occ, sc_bbox(g));
    }
    hipLaunchKernelGGL(k_pose_bins, dim3((P + 63) / 64), dim3(64), 0, st, g->poses, P, sc_bbox(g), n_occ);
    hipLaunchKernelGGL(k_fill_i32, dim3(1024), dim3(256), 0, st, g->counts, g->bin_total, 0);
    const unsigned occ_blk = (unsigned)std::max<int64_t>(1, (n_occ + 255) / 256);
    if (n_occ > 0)
        hipLaunchKernelGGL(k_bin_count, dim3(occ_blk, P), dim3(256), 0, st, g->poses, g->verts, N, g->list, n_occ, g->counts);
    hipLaunchKernelGGL(k_scan, dim3(P), dim3(1024), 0, st, g->poses, g->counts, g->bin_start, sc_totals(g));
    hipLaunchKernelGGL(k_ref_offsets, dim3(1), dim3(64), 0, st, g->poses, P, sc_totals(g), fill ? g->ref_capacity : (int64_t)0,
                       sc_overflow(g));
    if (fill && n_occ > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1024), dim3(256), 0, st, g->counts, g->bin_total, 0);
        hipLaunchKernelGGL(k_bin_fill, dim3(occ_blk, P), dim3(256), 0, st, g->poses, g->verts, N, g->list, n_occ,
                           g->bin_start, g->counts, g->bin_cells);
        hipLaunchKernelGGL(k_bin_sort, dim3((unsigned)((g->max_bins + 255) / 256), P), dim3(256), 0, st, g->poses,
                           g->bin_start, g->bin_cells);
    }
    return check_hip(hipGetLastError(), "grid rebin launch");
}

static void set_pose_params(std::vector<PoseDev>& P, const nif_pose* poses) {
    for (size_t p = 0; p < P.size(); ++p) {
        P[p].kind = poses[p].kind;
        P[p].s = poses[p].strength;
        pose_constants(P[p].kind, P[p].s, &P[p].k0, &P[p].k1, &P[p].k2);
    }
}

int grid_build(nif_grid* g, const uint8_t* occ, int32_t N, const nif_pose* poses, int32_t n_poses,
               int32_t bins_per_axis, hipStream_t st) {
    g->N = N;
    g->n_poses = n_poses;
    const int64_t nv = (int64_t)(N + 1) * (N + 1) * (N + 1);
    const int64_t ncell = (int64_t)N * N * N;
    const int nbin_axis = bins_per_axis > 0 ? bins_per_axis : (N / 2 > 0 ? N / 2 : 1);
    std::vector<PoseDev> P(n_poses);
    for (int p = 0; p < n_poses; ++p) {
        memset(&P[p], 0, sizeof(PoseDev));
        P[p].vert_off = nv * p;
        P[p].nb[0] = P[p].nb[1] = P[p].nb[2] = 1;
    }
    set_pose_params(P, poses);
    int rc;
#define NIF_TRY(expr, what)                                      \
    do {                                                         \
        if ((rc = check_hip((expr), what)) != NIF_OK) return rc; \
    } while (0)
    NIF_TRY(hipMalloc(&g->poses, sizeof(PoseDev) * n_poses), "hipMalloc poses");
    NIF_TRY(hipMalloc(&g->verts, sizeof(float4) * nv * n_poses), "hipMalloc vertices");
    NIF_TRY(hipMalloc(&g->scratch, sizeof(int32_t) * (7 * n_poses + 8)), "hipMalloc grid scratch");
    NIF_TRY(hipMalloc(&g->order_pre, sizeof(int64_t) * 8 * (n_poses + 1)), "hipMalloc dealing table");
    NIF_TRY(hipMalloc(&g->list, sizeof(int32_t) * (ncell + 1)), "hipMalloc occupied list");
    // occupied voxels, compacted once
    NIF_TRY(hipMemsetAsync(sc_nocc(g), 0, sizeof(int32_t), st), "memset");
    hipLaunchKernelGGL(k_compact, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, st, occ, ncell, g->list, sc_nocc(g));
    NIF_TRY(hipGetLastError(), "k_compact");
    int32_t n_occ = 0;
    NIF_TRY(hipMemcpyAsync(&n_occ, sc_nocc(g), sizeof(int32_t), hipMemcpyDeviceToHost, st), "read count");
    NIF_TRY(hipStreamSynchronize(st), "sync");
    g->n_occupied = n_occ;
    // the first poses' bounding boxes fix the bins per axis (by aspect ratio)
    NIF_TRY(hipMemcpyAsync(g->poses, P.data(), sizeof(PoseDev) * n_poses, hipMemcpyHostToDevice, st), "copy poses");
    hipLaunchKernelGGL(k_vertices, dim3((unsigned)((nv + 255) / 256), n_poses), dim3(256), 0, st, g->poses, N, g->verts);
    hipLaunchKernelGGL(k_bbox_init, dim3((6 * n_poses + 255) / 256), dim3(256), 0, st, sc_bbox(g), n_poses);
    if (n_occ > 0) {
        unsigned nblk = (unsigned)std::min<int64_t>((n_occ + 255) / 256, 1024);
        hipLaunchKernelGGL(k_pose_bbox, dim3(nblk, n_poses), dim3(256), 0, st, g->poses, g->verts, N, g->list, n_occ, sc_bbox(g));
    }
    NIF_TRY(hipGetLastError(), "bbox");
    std::vector<int32_t> bb(6 * n_poses);
    NIF_TRY(hipMemcpyAsync(bb.data(), sc_bbox(g), sizeof(int32_t) * 6 * n_poses, hipMemcpyDeviceToHost, st), "read bbox");
    NIF_TRY(hipStreamSynchronize(st), "sync");
    int64_t bin_total = 0, max_bins = 1;
    for (int p = 0; p < n_poses; ++p) {
        float e[3], ext = 0.f;
        for (int c = 0; c < 3; ++c) {
            e[c] = n_occ == 0 ? 1.f : ord2f_host(bb[6 * p + 3 + c]) - ord2f_host(bb[6 * p + c]);
            ext = std::max(ext, e[c]);
        }
        for (int c = 0; c < 3; ++c) P[p].nb[c] = std::max(1, std::min((int)std::ceil(nbin_axis * e[c] / ext - 1e-3f), 4096));
        P[p].bin_off = bin_total;
        const int64_t nb = (int64_t)P[p].nb[0] * P[p].nb[1] * P[p].nb[2];
        bin_total += nb + 1;
        max_bins = std::max(max_bins, nb);
    }
    g->bin_total = bin_total;
    g->max_bins = max_bins;
    NIF_TRY(hipMalloc(&g->bin_start, sizeof(int32_t) * bin_total), "hipMalloc bin_start");
    NIF_TRY(hipMalloc(&g->counts, sizeof(int32_t) * bin_total), "hipMalloc bin counts");
    NIF_TRY(hipMemcpyAsync(g->poses, P.data(), sizeof(PoseDev) * n_poses, hipMemcpyHostToDevice, st), "copy poses");
    // count pass, then size the reference lists with headroom for later re-poses
    g->ref_capacity = 0;
    if ((rc = grid_rebin(g, false, st))) return rc;
    std::vector<int32_t> tot(n_poses);
    NIF_TRY(hipMemcpyAsync(tot.data(), sc_totals(g), sizeof(int32_t) * n_poses, hipMemcpyDeviceToHost, st), "read totals");
    NIF_TRY(hipStreamSynchronize(st), "sync");
    int64_t refs = 0;
    for (int p = 0; p < n_poses; ++p) refs += tot[p];
    g->ref_capacity = refs + refs / 2 + 4096;
    NIF_TRY(hipMalloc(&g->bin_cells, sizeof(int32_t) * g->ref_capacity), "hipMalloc bin_cells");
    if ((rc = grid_rebin(g, true, st))) return rc;
    NIF_TRY(hipStreamSynchronize(st), "sync");
    g->poses_host = P;
    g->refs_per_pose.assign(tot.begin(), tot.end());
#undef NIF_TRY
    return NIF_OK;
}

int grid_update(nif_grid* g, const nif_pose* poses, hipStream_t st) {
    set_pose_params(g->poses_host, poses);
    // kind, strength and constants change; boxes, bin sizes and offsets are recomputed on the device
    int rc = check_hip(hipMemcpyAsync(g->poses, g->poses_host.data(), sizeof(PoseDev) * g->n_poses,
                                      hipMemcpyHostToDevice, st), "copy poses");
    if (rc) return rc;
    return grid_rebin(g, true, st);
}

int grid_bounds(const nif_grid* g, int pose, float* lo, float* hi) {
    PoseDev pd;
    int rc = check_hip(hipMemcpy(&pd, g->poses + pose, sizeof(PoseDev), hipMemcpyDeviceToHost), "read pose");
    if (rc) return rc;
    for (int a = 0; a < 3; ++a) {
        lo[a] = pd.empty ? 0.f : pd.lo[a];
        hi[a] = pd.empty ? 0.f : pd.lo[a] + pd.bs[a] * (float)pd.nb[a];
    }
    return NIF_OK;
}

int grid_overflow(nif_grid* g, hipStream_t st, int32_t* overflow) {
    int rc = check_hip(hipMemcpyAsync(overflow, sc_overflow(g), sizeof(int32_t), hipMemcpyDeviceToHost, st), "read overflow");
    if (rc) return rc;
    return check_hip(hipStreamSynchronize(st), "sync");
}

}  // namespace nif
