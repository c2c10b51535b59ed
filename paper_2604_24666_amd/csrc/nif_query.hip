// Query-side kernels: segment tracing, the fused first-hit query, the voxel proxy, and the
// network on given rest-space points.
//
// The fused query (Methodology; "Segmented Ray Distance Accumulation") is one persistent
// kernel.  Every lane owns a ray; a wave takes rays from a global counter (one atomic per
// wave, rays of all poses in one index space).  Each round, every lane finds its ray's next
// occupied deformed voxel, maps the voxel's entry/exit points to rest space, and the wave
// evaluates encoding + MLP for all 64 segments together on MFMA.  A lane whose hit logit is
// positive writes the ray's result and takes a new ray; the others continue front to back.
// Lanes whose rays miss everything take new rays before the network round, so the MFMA
// tiles stay full while rays last.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "nif_internal.hpp"
#include "nif_net.hpp"
#include "nif_trace.hpp"

namespace nif {

struct GridArgs {
    const PoseDev* poses;
    const float4* V;
    const int32_t* bin_start;
    const int32_t* bin_cells;
    int32_t N;
};

struct RayArgs {
    const float *ox, *oy, *oz, *dx, *dy, *dz;
    const int64_t* off;
    const float* tmax;          // nullable: occlusion bound per ray
    int32_t n_poses;
    int64_t n;
    const int64_t* order_pre;   // nullable: pose-ordered dealing, [8][n_poses + 1] (k_order_prefix)
};

__device__ __forceinline__ Ray load_ray(const RayArgs& R, int64_t r) {
    Ray ray;
    ray.o = make_float3(R.ox[r], R.oy[r], R.oz[r]);
    ray.d = make_float3(R.dx[r], R.dy[r], R.dz[r]);
    return ray;
}

__device__ __forceinline__ float3 ray_at(const Ray& R, float t) {
    return make_float3(fmaf(t, R.d.x, R.o.x), fmaf(t, R.d.y, R.o.y), fmaf(t, R.d.z, R.o.z));
}

__global__ void k_reset(int64_t* counters, int n) {
    if (threadIdx.x < n) counters[threadIdx.x] = 0;
}

// Per-pose timing slots of the stats buffer: [4] start (min over waves), [5, 5+P) completion
// time of each pose, [5+P, 5+2P) rays finished per pose.
__global__ void k_reset_pose_times(int64_t* stats, int n_poses) {
    for (int i = threadIdx.x; i < 1 + 2 * n_poses; i += blockDim.x) stats[4 + i] = i == 0 ? INT64_MAX : 0;
}

// Counts finished rays per pose (one atomic per wave when the finishing lanes share a pose)
// and stamps a pose's completion time when its last ray is done.  Called by the whole wave.
__device__ __forceinline__ void note_finished(int64_t* stats, const int64_t* off, int n_poses, bool fin, int pose) {
    const uint64_t m = ballot(fin);
    if (!m) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int p0 = __shfl(pose, leader);
    const bool uniform = ballot(fin && pose != p0) == 0;
    int64_t* done = stats + 5 + n_poses;
    if (uniform) {
        if (lane_id() == leader) {
            const int64_t total = off[p0 + 1] - off[p0];
            const int64_t c = (int64_t)popc64(m);
            const int64_t old = (int64_t)atomicAdd((unsigned long long*)&done[p0], (unsigned long long)c);
            if (old + c == total) atomicMax((unsigned long long*)&stats[5 + p0], (unsigned long long)wall_clock64());
        }
    } else if (fin) {
        const int64_t total = off[pose + 1] - off[pose];
        const int64_t old = (int64_t)atomicAdd((unsigned long long*)&done[pose], 1ull);
        if (old + 1 == total) atomicMax((unsigned long long*)&stats[5 + pose], (unsigned long long)wall_clock64());
    }
}

// ------------------------------------------------------------------ segments of every ray

__global__ void __launch_bounds__(256) k_trace(GridArgs G, RayArgs R, int32_t max_seg, nif_segments out) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R.n; r += (int64_t)gridDim.x * blockDim.x) {
        const Ray ray = load_ray(R, r);
        const PoseDev P = G.poses[find_pose(R.off, R.n_poses, r)];
        Trav tv;
        trav_init(P, ray, tv);
        Segment sg;
        int bad = 0, n = 0;
        const int64_t total = R.n * (int64_t)max_seg;
        while (next_segment(P, G.V, G.bin_start, G.bin_cells, G.N, ray, tv, sg, &bad)) {
            if (n < max_seg) {
                const int64_t k = r * max_seg + n;
                if (out.cell) out.cell[k] = sg.cell;
                if (out.t_in) out.t_in[k] = sg.a;
                if (out.t_out) out.t_out[k] = sg.b;
                if (out.x0 || out.x1) {
                    const float3 x0 = deform_inv(P, ray_at(ray, sg.a));
                    const float3 x1 = deform_inv(P, ray_at(ray, sg.b));
                    if (out.x0) { out.x0[k] = x0.x; out.x0[total + k] = x0.y; out.x0[2 * total + k] = x0.z; }
                    if (out.x1) { out.x1[k] = x1.x; out.x1[total + k] = x1.y; out.x1[2 * total + k] = x1.z; }
                }
            }
            ++n;
        }
        if (out.count) out.count[r] = n;
    }
}

// ------------------------------------------------------------------ outputs of one ray

__device__ __forceinline__ void write_miss(const nif_hits& o, int64_t r, int nq, float last_z0) {
    if (o.hit) o.hit[r] = 0;
    if (o.t) o.t[r] = INFINITY;
    if (o.nx) o.nx[r] = 0.f;
    if (o.ny) o.ny[r] = 0.f;
    if (o.nz) o.nz[r] = 0.f;
    if (o.ar) o.ar[r] = 0.f;
    if (o.ag) o.ag[r] = 0.f;
    if (o.ab) o.ab[r] = 0.f;
    if (o.material) o.material[r] = -1;
    if (o.cell) o.cell[r] = -1;
    if (o.hit_logit) o.hit_logit[r] = last_z0;
    if (o.n_queried) o.n_queried[r] = nq;
    if (o.xr) o.xr[r] = 0.f;
    if (o.yr) o.yr[r] = 0.f;
    if (o.zr) o.zr[r] = 0.f;
    if (o.dnx) o.dnx[r] = 0.f;
    if (o.dny) o.dny[r] = 0.f;
    if (o.dnz) o.dnz[r] = 0.f;
}

__device__ __forceinline__ float sigmoidf_(float v) { return 1.f / (1.f + expf(-v)); }

// Writes the hit of segment sg; a hit at or beyond tmax is written as a miss instead.
__device__ __forceinline__ void write_hit(const nif_hits& o, int64_t r, const Segment& sg, float3 x0, float3 x1,
                                          const float* z, int nq, int n_mat, int dist_head, float tmax,
                                          const PoseDev& P) {
    const float ex = x1.x - x0.x, ey = x1.y - x0.y, ez = x1.z - x0.z;
    float f;
    if (dist_head == NIF_DIST_SIGMOID) {
        f = sigmoidf_(z[1]);               // the bounded head: the fraction itself
    } else {
        const float lr = sqrtf(ex * ex + ey * ey + ez * ez);
        const float dh = fmaxf(z[1], 0.f);
        f = lr > 0.f ? fminf(fmaxf(dh / lr, 0.f), 1.f) : 0.f;
    }
    const float D = fmaf(f, sg.b - sg.a, sg.a);
    if (D >= tmax) {
        write_miss(o, r, nq, z[0]);
        return;
    }
    if (o.hit) o.hit[r] = 1;
    if (o.t) o.t[r] = D;
    const float nl = fmaxf(sqrtf(z[2] * z[2] + z[3] * z[3] + z[4] * z[4]), 1e-12f);
    if (o.nx) o.nx[r] = z[2] / nl;
    if (o.ny) o.ny[r] = z[3] / nl;
    if (o.nz) o.nz[r] = z[4] / nl;
    if (o.ar) o.ar[r] = sigmoidf_(z[5]);
    if (o.ag) o.ag[r] = sigmoidf_(z[6]);
    if (o.ab) o.ab[r] = sigmoidf_(z[7]);
    if (o.material) {
        int best = 0;
        if (n_mat == 1) best = z[8] > 0.f ? 1 : 0;
        else
            for (int c = 1; c < n_mat; ++c)
                if (z[8 + c] > z[8 + best]) best = c;
        o.material[r] = best;
    }
    if (o.cell) o.cell[r] = sg.cell;
    if (o.hit_logit) o.hit_logit[r] = z[0];
    if (o.n_queried) o.n_queried[r] = nq;
    if (o.xr) o.xr[r] = fmaf(f, ex, x0.x);
    if (o.yr) o.yr[r] = fmaf(f, ey, x0.y);
    if (o.zr) o.zr[r] = fmaf(f, ez, x0.z);
    if (o.dnx || o.dny || o.dnz) {
        const float3 xh = make_float3(fmaf(f, ex, x0.x), fmaf(f, ey, x0.y), fmaf(f, ez, x0.z));
        const float3 dn = deform_normal(P, xh, make_float3(z[2] / nl, z[3] / nl, z[4] / nl));
        if (o.dnx) o.dnx[r] = dn.x;
        if (o.dny) o.dny[r] = dn.y;
        if (o.dnz) o.dnz[r] = dn.z;
    }
}

__device__ __forceinline__ void wave_add_stats(int64_t* stats, int64_t a, int64_t b, int64_t c) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
    if (lane_id() == 0) {
        atomicAdd((unsigned long long*)&stats[0], (unsigned long long)a);
        atomicAdd((unsigned long long*)&stats[1], (unsigned long long)b);
        atomicAdd((unsigned long long*)&stats[2], (unsigned long long)c);
    }
}

// ------------------------------------------------------------------ fused first-hit query
//
// Register budget.  The traversal state of a lane (ray index, pose, DDA state, current
// segment) is parked in LDS while the wave runs the network, so the encoding + MLP phase
// holds only its own values and the kernel fits more waves per SIMD; the ray and the pose
// constants are re-read (L1/L2 resident) when the lane resumes.  One wave per workgroup.

// Parked words per lane, stored [word][64] (lane-consecutive, no bank conflicts).
enum {
    QW_R_LO, QW_R_HI, QW_POSE, QW_NQ, QW_LASTZ, QW_HAS,
    QW_IX, QW_IY, QW_IZ, QW_TMX, QW_TMY, QW_TMZ, QW_TDX, QW_TDY, QW_TDZ, QW_EX, QW_EY, QW_EZ,
    QW_SX, QW_SY, QW_SZ, QW_TLO, QW_LASTA, QW_LASTC, QW_ACTIVE,
    QW_CELL, QW_A, QW_B,
    QW_WORDS
};

struct Parked {
    int32_t* w;
    int lane;
    __device__ __forceinline__ void put(int k, int32_t v) const { w[k * 64 + lane] = v; }
    __device__ __forceinline__ void putf(int k, float v) const { w[k * 64 + lane] = __float_as_int(v); }
    __device__ __forceinline__ int32_t get(int k) const { return w[k * 64 + lane]; }
    __device__ __forceinline__ float getf(int k) const { return __int_as_float(w[k * 64 + lane]); }
};

__device__ __forceinline__ void park_trav(const Parked& pk, const Trav& T) {
    pk.put(QW_IX, T.ix); pk.put(QW_IY, T.iy); pk.put(QW_IZ, T.iz);
    pk.putf(QW_TMX, T.tmx); pk.putf(QW_TMY, T.tmy); pk.putf(QW_TMZ, T.tmz);
    pk.putf(QW_TDX, T.tdx); pk.putf(QW_TDY, T.tdy); pk.putf(QW_TDZ, T.tdz);
    pk.put(QW_EX, T.ex); pk.put(QW_EY, T.ey); pk.put(QW_EZ, T.ez);
    pk.put(QW_SX, T.sx); pk.put(QW_SY, T.sy); pk.put(QW_SZ, T.sz);
    pk.putf(QW_TLO, T.t_lo); pk.putf(QW_LASTA, T.last_a); pk.put(QW_LASTC, T.last_cell); pk.put(QW_ACTIVE, T.active);
}

__device__ __forceinline__ void unpark_trav(const Parked& pk, Trav& T) {
    T.ix = pk.get(QW_IX); T.iy = pk.get(QW_IY); T.iz = pk.get(QW_IZ);
    T.tmx = pk.getf(QW_TMX); T.tmy = pk.getf(QW_TMY); T.tmz = pk.getf(QW_TMZ);
    T.tdx = pk.getf(QW_TDX); T.tdy = pk.getf(QW_TDY); T.tdz = pk.getf(QW_TDZ);
    T.ex = pk.get(QW_EX); T.ey = pk.get(QW_EY); T.ez = pk.get(QW_EZ);
    T.sx = pk.get(QW_SX); T.sy = pk.get(QW_SY); T.sz = pk.get(QW_SZ);
    T.t_lo = pk.getf(QW_TLO); T.last_a = pk.getf(QW_LASTA); T.last_cell = pk.get(QW_LASTC); T.active = pk.get(QW_ACTIVE);
}

#ifndef NIF_QUERY_MIN_WAVES
#define NIF_QUERY_MIN_WAVES 2
#endif

// RPW rays per wave (64, or 16 for launches too small to hide the latency of a network round:
// then a round is one pass of 16 segments instead of four, and four times as many waves run).
template <int HW, int PREC, int RPW, bool GAMMA = false, int FD = 2>
__global__ void __launch_bounds__(64, NIF_QUERY_MIN_WAVES) k_query(NetParams np, GridArgs G, RayArgs R, nif_hits out,
                                              int64_t* __restrict__ counters, int64_t* __restrict__ stats,
                                              int pose_times) {
    static_assert(RPW == 16 || RPW == 64, "rays per wave");
    constexpr int CB = kQueryCB;
    constexpr int PASSES = RPW / 16 / CB;
    __shared__ int32_t s_park[QW_WORDS * 64];
    __shared__ float s_seg[64 * kSegStride];
    __shared__ float s_z[64 * kZStride];
    const int lane = lane_id();
    const Parked pk{s_park, lane};
    const int n_mat = np.H - 8;

    // Rays are dealt in 8 contiguous ranges, one per XCD: workgroups are dispatched to the
    // XCDs round-robin, so workgroup b starts on range b mod 8 and the waves sharing an L2
    // walk neighbouring rays (coherent rays touch the same table lines).  A wave whose range
    // runs dry moves on to the next one, so the load still balances across the chip.  With
    // pose-ordered dealing, range k is the concatenation over the poses of the k-th eighth of
    // each pose's rays (positions counted in R.order_pre), so every XCD finishes pose p
    // before it starts pose p + 1.
    const int home = (int)(blockIdx.x & 7);
    const int64_t span = (R.n + 7) / 8;
    const int64_t* opre = R.order_pre;
    auto range_of = [&](int id, int64_t& l, int64_t& h) {
        if (opre) {
            l = 0;
            h = opre[(int64_t)id * (R.n_poses + 1) + R.n_poses];
        } else {
            l = std::min<int64_t>((int64_t)id * span, R.n);
            h = std::min<int64_t>(l + span, R.n);
        }
    };
    int cur = 0;                                   // ranges tried (wave-uniform); 8 = none left
    int rid = home;
    int64_t lo, hi;
    range_of(rid, lo, hi);
    int bad = 0;
    int64_t n_done = 0, n_eval = 0;
    if (pose_times && lane == 0) atomicMin((unsigned long long*)&stats[4], (unsigned long long)wall_clock64());
    pk.put(QW_R_LO, -1); pk.put(QW_R_HI, -1); pk.put(QW_HAS, 0); pk.put(QW_POSE, 0);

    for (;;) {
        // ---- resume the lane: ray, pose, and the result of the last network round
        int64_t r = (int64_t)(((uint64_t)(uint32_t)pk.get(QW_R_HI) << 32) | (uint32_t)pk.get(QW_R_LO));
        int pose = pk.get(QW_POSE);
        bool has = pk.get(QW_HAS) != 0;
        int nq = 0;
        float last_z0 = -INFINITY;
        Ray ray;
        ray.o = ray.d = make_float3(0.f, 0.f, 0.f);
        Trav tv;
        tv.active = 0;
        PoseDev P;
        P.kind = 0;
        Segment sg;
        sg.cell = -1; sg.a = sg.b = 0.f; sg.face = -1;
        if (r >= 0) {
            nq = pk.get(QW_NQ);
            last_z0 = pk.getf(QW_LASTZ);
            unpark_trav(pk, tv);
            ray = load_ray(R, r);
            P = G.poses[pose];
        }
        bool hitnow = false;
        if (has) {
            ++nq;
            ++n_eval;
            const float* z = s_z + lane * kZStride;
            last_z0 = z[0];
            if (z[0] > 0.f) {
                sg.cell = pk.get(QW_CELL); sg.a = pk.getf(QW_A); sg.b = pk.getf(QW_B);
                const float* my = s_seg + lane * kSegStride;
                write_hit(out, r, sg, make_float3(my[0], my[1], my[2]), make_float3(my[4], my[5], my[6]), z, nq, n_mat,
                          np.dist_head, R.tmax ? R.tmax[r] : INFINITY, P);
                r = -1;
                ++n_done;
                hitnow = true;
            }
            has = false;
        }
        if (pose_times) note_finished(stats, R.off, R.n_poses, hitnow, pose);

        // ---- give every lane a segment, taking new rays as old ones finish or miss
        for (;;) {
            const bool need = cur < 8 && r < 0 && lane < RPW;
            const uint64_t m = ballot(need);
            if (m) {
                const int leader = __ffsll((unsigned long long)m) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd((unsigned long long*)&counters[rid], (unsigned long long)popc64(m));
                base = __shfl(base, leader);
                if (need) {
                    r = lo + (int64_t)base + rank_below(m);
                    if (r >= hi) {
                        r = -1;
                    } else {
                        if (opre) {                  // position r of range rid -> (pose, ray)
                            const int64_t* pre = opre + (int64_t)rid * (R.n_poses + 1);
                            int a = 0, b = R.n_poses - 1;
                            while (a < b) {          // last pose p with pre[p] <= r
                                const int mid = (a + b + 1) >> 1;
                                if (pre[mid] <= r) a = mid; else b = mid - 1;
                            }
                            pose = a;
                            const int64_t cnt = R.off[a + 1] - R.off[a];
                            r = R.off[a] + cnt * rid / 8 + (r - pre[a]);
                        } else {
                            pose = find_pose(R.off, R.n_poses, r);
                        }
                        ray = load_ray(R, r);
                        P = G.poses[pose];
                        trav_init(P, ray, tv);
                        nq = 0;
                        last_z0 = -INFINITY;
                    }
                }
                if (lo + (int64_t)base + popc64(m) >= hi) {       // this range is used up: next one
                    ++cur;
                    rid = (home + cur) & 7;
                    range_of(rid, lo, hi);
                }
            }
            const bool search = r >= 0 && !has;
            if (!ballot(search)) {
                if (cur < 8 && ballot(r < 0 && lane < RPW)) continue;   // lanes still to fill
                break;
            }
            bool missed = false;
            if (search) {
                has = next_segment(P, G.V, G.bin_start, G.bin_cells, G.N, ray, tv, sg, &bad);
                if (has && R.tmax && sg.a >= R.tmax[r]) has = false;     // occlusion bound reached
                if (!has) {
                    write_miss(out, r, nq, last_z0);
                    r = -1;
                    ++n_done;
                    missed = true;
                }
            }
            if (pose_times) note_finished(stats, R.off, R.n_poses, missed, pose);
        }
        if (!ballot(has)) break;

        // ---- rest-space entry/exit points (local linearization inside the voxel), park, network
        float3 x0 = make_float3(0.5f, 0.5f, 0.5f), x1 = x0;
        if (has) {
            x0 = deform_inv(P, ray_at(ray, sg.a));
            x1 = deform_inv(P, ray_at(ray, sg.b));
        }
        float* my = s_seg + lane * kSegStride;
        my[0] = x0.x; my[1] = x0.y; my[2] = x0.z;
        my[4] = x1.x; my[5] = x1.y; my[6] = x1.z;
        pk.put(QW_R_LO, (int32_t)(uint32_t)(uint64_t)r); pk.put(QW_R_HI, (int32_t)(uint32_t)((uint64_t)r >> 32));
        pk.put(QW_POSE, pose); pk.put(QW_HAS, has ? 1 : 0);
        if (r >= 0) {
            pk.put(QW_NQ, nq); pk.putf(QW_LASTZ, last_z0);
            park_trav(pk, tv);
            pk.put(QW_CELL, sg.cell); pk.putf(QW_A, sg.a); pk.putf(QW_B, sg.b);
        }
        wave_lds_sync();
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) net_pass<HW, CB, PREC, GAMMA, FD>(np, s_seg, ps * 16 * CB, s_z, nullptr, 0, 0, 0);
        wave_lds_sync();
    }
    if (stats) wave_add_stats(stats, n_done, n_eval, bad);
}

// ------------------------------------------------------------------ voxel proxy (no network)
// The first occupied voxel is the hit: D = t_in, rest point D^-1(entry), normal = outward
// rest-space normal of the entered face.

__global__ void __launch_bounds__(256) k_proxy(GridArgs G, RayArgs R, nif_hits out, int64_t* __restrict__ stats) {
    int64_t n_done = 0;
    int bad = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R.n; r += (int64_t)gridDim.x * blockDim.x) {
        const Ray ray = load_ray(R, r);
        const PoseDev P = G.poses[find_pose(R.off, R.n_poses, r)];
        Trav tv;
        trav_init(P, ray, tv);
        Segment sg;
        const float tmax = R.tmax ? R.tmax[r] : INFINITY;
        if (next_segment(P, G.V, G.bin_start, G.bin_cells, G.N, ray, tv, sg, &bad) && sg.a < tmax) {
            const float3 x0 = deform_inv(P, ray_at(ray, sg.a));
            float z[16];
            for (int i = 0; i < 16; ++i) z[i] = 0.f;
            z[0] = 1.f;
            // the face normal enters the outputs as z_n; the distance head is 0 so D = t_in
            if (sg.face >= 0) z[2 + (sg.face >> 1)] = (sg.face & 1) ? 1.f : -1.f;
            write_hit(out, r, sg, x0, x0, z, 1, 1, NIF_DIST_LOG_RELU, tmax, P);
            if (out.ar) out.ar[r] = 0.f;
            if (out.ag) out.ag[r] = 0.f;
            if (out.ab) out.ab[r] = 0.f;
            if (out.material) out.material[r] = 0;
        } else {
            write_miss(out, r, 0, -INFINITY);
        }
        ++n_done;
    }
    if (stats) {
        int64_t a = n_done, c = bad;
        for (int off = 32; off > 0; off >>= 1) { a += __shfl_xor(a, off); c += __shfl_xor(c, off); }
        if (lane_id() == 0) {
            atomicAdd((unsigned long long*)&stats[0], (unsigned long long)a);
            atomicAdd((unsigned long long*)&stats[2], (unsigned long long)c);
        }
    }
}

// ------------------------------------------------------------------ network on given points

// Full encoding of n points (lane per point): out[i][(s L + l) Fd + f].
__global__ void __launch_bounds__(256) k_encode(EncParams ep, const float* __restrict__ x, int64_t n,
                                                float* __restrict__ out) {
    const int S = 1 + 2 * ep.F;
    const int W = S * ep.L * ep.Fd;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        PEState pe;
        pe_begin(pe, x[i], x[n + i], x[2 * n + i]);
        for (int s = 0; s < S; ++s) {
            double smp[3];
            pe_sample(pe, s, smp);
            for (int l = 0; l < ep.L; ++l) {
                float* o = out + i * W + (s * ep.L + l) * ep.Fd;
                if (ep.f16) grid_lookup_any<true>(ep, l, smp[0], smp[1], smp[2], set_offset(ep, s), o);
                else grid_lookup_any<false>(ep, l, smp[0], smp[1], smp[2], set_offset(ep, s), o);
            }
        }
    }
}

// Encoding of segments [seg_base, seg_base + 16*CB) into enc_out only (no MLP past the
// first layer's accumulation, whose result is dropped).
template <int HW, int CB, int PREC, bool GAMMA, int FD>
__device__ __forceinline__ void enc_pass(const NetParams& np, const float* s_seg, int seg_base, int64_t seg_g0,
                                         int64_t n_valid, float* enc_out) {
    floatx4 acc[HW / 16][CB];
    layer1_bias<HW, CB>(np, acc);
    layer1_levels<HW, CB, PREC, FD>(np, s_seg, seg_base, 0, np.enc.L, acc, enc_out, seg_g0, n_valid);
    if constexpr (GAMMA) layer1_gamma<HW, CB, PREC>(np, s_seg, seg_base, acc, enc_out, seg_g0, n_valid);
}

// Heads of point pairs.  Each wave evaluates tiles of 64 pairs; acts (nullable) receives the
// hidden activations [layer][B][HW] and enc (nullable) the encoding [B][E], for the training
// backward.  x0 / x1 are SoA with row stride ld >= B.  ENC_ONLY: only the encoding is written
// (the backward's recomputation, per chunk of samples; heads and acts unused), in tiles of 16
// pairs so that a chunk still spreads over many waves.  At width 128 each pass takes 16 of
// the tile's 64 points, which keeps the accumulators small enough for two waves per SIMD; with
// spatially ordered batches that latency hiding outweighs streaming the first-layer weights
// once per pass.
template <int HW, int PREC, bool GAMMA = false, bool ENC_ONLY = false, int TILE = ENC_ONLY ? 16 : 64, int FD = 2>
__global__ void __launch_bounds__(256, 2) k_forward(NetParams np, const float* __restrict__ x0, const float* __restrict__ x1,
                                                 int64_t B, int64_t ld, float* __restrict__ heads,
                                                 float* __restrict__ acts, float* __restrict__ enc) {
    constexpr int CB = TILE == 16 || HW >= 128 ? 1 : 4;
    constexpr int PASSES = TILE / 16 / CB;
    __shared__ float s_seg_all[4][64 * kSegStride];
    __shared__ float s_z_all[4][64 * kZStride];
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    float* s_seg = s_seg_all[w];
    float* s_z = s_z_all[w];
    const int64_t n_tiles = (B + TILE - 1) / TILE;
    const int64_t wave_g = (int64_t)blockIdx.x * 4 + w, n_waves = (int64_t)gridDim.x * 4;
    for (int64_t tile = wave_g; tile < n_tiles; tile += n_waves) {
        const int64_t seg = tile * TILE + lane;
        float* my = s_seg + lane * kSegStride;
        if (lane < TILE && seg < B) {
            my[0] = x0[seg]; my[1] = x0[ld + seg]; my[2] = x0[2 * ld + seg];
            my[4] = x1[seg]; my[5] = x1[ld + seg]; my[6] = x1[2 * ld + seg];
        } else {
            my[0] = my[1] = my[2] = my[4] = my[5] = my[6] = 0.5f;
        }
        wave_lds_sync();
        if constexpr (ENC_ONLY) {
#pragma unroll
            for (int ps = 0; ps < PASSES; ++ps)
                enc_pass<HW, CB, PREC, GAMMA, FD>(np, s_seg, ps * 16 * CB, tile * TILE + ps * 16 * CB, B, enc);
        } else {
#pragma unroll
            for (int ps = 0; ps < PASSES; ++ps)
                net_pass<HW, CB, PREC, GAMMA, FD>(np, s_seg, ps * 16 * CB, s_z, acts, B * HW, tile * TILE + ps * 16 * CB, B, enc);
            wave_lds_sync();
            if (lane < TILE && seg < B)
                for (int h = 0; h < np.H; ++h) heads[seg * np.H + h] = s_z[lane * kZStride + h];
        }
        wave_lds_sync();
    }
}

// ------------------------------------------------------------------ host launchers

static int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

NetParams make_net_params(const nif_model* m, int32_t precision) {
    NetParams np;
    memset(&np, 0, sizeof(np));
    const nif_model_desc& d = m->desc;
    np.enc.tab = d.table_dtype == NIF_TABLE_F16 ? (const void*)m->tables_h : (const void*)m->tables;
    np.enc.f16 = d.table_dtype == NIF_TABLE_F16;
    np.enc.L = d.levels;
    np.enc.Fd = d.feat_dim;
    np.enc.log2T = d.log2_table;
    np.enc.F = d.concat_encoding ? 0 : d.pe_freqs;      // the grid sees x only in the concatenated form
    np.gamma_F = d.concat_encoding ? d.pe_freqs : -1;
    np.E_phi = 2 * m->S * d.levels * d.feat_dim;
    np.enc.dense_mask = 0;
    np.enc.set_stride = d.per_sample_tables ? ((int64_t)d.levels << d.log2_table) : 0;
    for (int l = 0; l < d.levels; ++l) {
        np.enc.res[l] = d.res[l];
        const uint64_t n1 = (uint64_t)d.res[l] + 1;
        if (n1 * n1 * n1 <= (1ull << d.log2_table)) np.enc.dense_mask |= 1u << l;
    }
    for (int i = 0; i < m->n_layers; ++i) {
        if (precision == NIF_PREC_FP32) np.W[i] = m->mlp_pad_f32 + m->wp_off[i];
        else if (precision == NIF_PREC_BF16) np.W[i] = m->mlp_pad_bf16 + m->wp_off[i];
        else np.W[i] = m->mlp_pad_f16 + m->wp_off[i];
        np.b[i] = m->mlp_pad_f32 + m->bp_off[i];
    }
    np.W0L = precision == NIF_PREC_FP32 ? (const void*)m->w0l_f32
           : precision == NIF_PREC_BF16 ? (const void*)m->w0l_bf16 : (const void*)m->w0l_f16;
    np.n_hidden = d.hidden_layers;
    np.E = m->E;
    np.H = m->H;
    np.dist_head = d.dist_head;
    return np;
}

static GridArgs grid_args(const nif_grid* g) {
    GridArgs G;
    G.poses = g->poses; G.V = g->verts; G.bin_start = g->bin_start; G.bin_cells = g->bin_cells; G.N = g->N;
    return G;
}

// Pose-ordered dealing: pre[k][p] = rays of poses 0 .. p-1 in range k, whose share of pose q
// is [off[q] + c_q k / 8, off[q] + c_q (k + 1) / 8), c_q the pose's ray count.
__global__ void k_order_prefix(const int64_t* __restrict__ off, int n_poses, int64_t* __restrict__ pre) {
    const int k = threadIdx.x;
    if (k >= 8) return;
    int64_t acc = 0;
    for (int p = 0; p < n_poses; ++p) {
        pre[(int64_t)k * (n_poses + 1) + p] = acc;
        const int64_t c = off[p + 1] - off[p];
        acc += c * (k + 1) / 8 - c * k / 8;
    }
    pre[(int64_t)k * (n_poses + 1) + n_poses] = acc;
}

static RayArgs ray_args(const nif_grid* g, const nif_rays* r, int64_t n) {
    RayArgs R;
    R.ox = r->ox; R.oy = r->oy; R.oz = r->oz; R.dx = r->dx; R.dy = r->dy; R.dz = r->dz;
    R.off = r->pose_offsets; R.tmax = r->tmax; R.n_poses = g->n_poses; R.n = n;
    R.order_pre = nullptr;
    return R;
}

int trace_launch(const nif_grid* g, const nif_rays* r, int64_t n, int32_t max_seg, const nif_segments* out,
                 hipStream_t st) {
    if (n == 0) return NIF_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)device_cus() * 16);
    hipLaunchKernelGGL(k_trace, dim3((unsigned)blocks), dim3(256), 0, st, grid_args(g), ray_args(g, r, n), max_seg, *out);
    return check_hip(hipGetLastError(), "k_trace launch");
}

// Persistent grid size of the fused query: one-wave workgroups per compute unit (tunable).
static int g_query_blocks_per_cu = 12;
// Rays per wave: 0 = by launch size, else 16 or 64.
static int g_query_rays_per_wave = 0;

// Below this many rays per compute unit a launch is latency-bound (the serial chain of
// network rounds of its longest rays sets the time), and 16-ray waves finish it sooner.
static constexpr int64_t kSmallLaunchRaysPerCU = 8192;

template <int HW, int PREC>
static void launch_query(const NetParams& np, const GridArgs& G, const RayArgs& R, const nif_hits& out, int64_t* ctr,
                         int64_t* stats, int pt, hipStream_t st) {
    int rpw = g_query_rays_per_wave;
    if (rpw == 0) rpw = R.n < kSmallLaunchRaysPerCU * device_cus() ? 16 : 64;
    const int64_t waves = (R.n + rpw - 1) / rpw;
    const int64_t blocks = std::max<int64_t>(std::min<int64_t>(waves, (int64_t)device_cus() * g_query_blocks_per_cu), 1);
    if (np.gamma_F >= 0 || np.enc.Fd == 3) {     // the method variants: one launch shape
        const int64_t b64 = std::max<int64_t>(std::min<int64_t>((R.n + 63) / 64, (int64_t)device_cus() * g_query_blocks_per_cu), 1);
        if (np.enc.Fd == 3)
            hipLaunchKernelGGL((k_query<HW, PREC, 64, false, 3>), dim3((unsigned)b64), dim3(64), 0, st, np, G, R, out, ctr, stats, pt);
        else
            hipLaunchKernelGGL((k_query<HW, PREC, 64, true>), dim3((unsigned)b64), dim3(64), 0, st, np, G, R, out, ctr, stats, pt);
    } else if (rpw == 16) {
        hipLaunchKernelGGL((k_query<HW, PREC, 16>), dim3((unsigned)blocks), dim3(64), 0, st, np, G, R, out, ctr, stats, pt);
    } else {
        hipLaunchKernelGGL((k_query<HW, PREC, 64>), dim3((unsigned)blocks), dim3(64), 0, st, np, G, R, out, ctr, stats, pt);
    }
}

template <int PREC>
static int dispatch_query(int hw, const NetParams& np, const GridArgs& G, const RayArgs& R, const nif_hits& out,
                          int64_t* ctr, int64_t* stats, int pt, hipStream_t st) {
    switch (hw) {
        case 16: launch_query<16, PREC>(np, G, R, out, ctr, stats, pt, st); break;
        case 32: launch_query<32, PREC>(np, G, R, out, ctr, stats, pt, st); break;
        case 64: launch_query<64, PREC>(np, G, R, out, ctr, stats, pt, st); break;
        case 128: launch_query<128, PREC>(np, G, R, out, ctr, stats, pt, st); break;
        default: return fail(NIF_E_UNSUPPORTED, "hidden_width must be 16, 32, 64 or 128");
    }
    return NIF_OK;
}

int query_launch(const nif_model* m, const nif_grid* g, const nif_rays* r, int64_t n, const nif_hits* out,
                 uint32_t flags, int32_t precision, int64_t* stats, hipStream_t st) {
    if (n == 0) return NIF_OK;
    const GridArgs G = grid_args(g);
    RayArgs R = ray_args(g, r, n);
    if (flags & NIF_Q_NO_NETWORK) {
        const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)device_cus() * 16);
        hipLaunchKernelGGL(k_proxy, dim3((unsigned)blocks), dim3(256), 0, st, G, R, *out, stats);
        return check_hip(hipGetLastError(), "k_proxy launch");
    }
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, m->counters, 8);
    if (flags & NIF_Q_POSE_ORDER) {
        hipLaunchKernelGGL(k_order_prefix, dim3(1), dim3(64), 0, st, R.off, R.n_poses, g->order_pre);
        R.order_pre = g->order_pre;
    }
    const int pt = (flags & NIF_Q_POSE_TIMES) && stats ? 1 : 0;
    if (pt) hipLaunchKernelGGL(k_reset_pose_times, dim3(1), dim3(256), 0, st, stats, g->n_poses);
    int rc;
    const NetParams np = make_net_params(m, precision);
    const int hw = m->desc.hidden_width;
    if (precision == NIF_PREC_FP32) rc = dispatch_query<P_FP32>(hw, np, G, R, *out, m->counters, stats, pt, st);
    else if (precision == NIF_PREC_BF16) rc = dispatch_query<P_BF16>(hw, np, G, R, *out, m->counters, stats, pt, st);
    else rc = dispatch_query<P_FP16>(hw, np, G, R, *out, m->counters, stats, pt, st);
    if (rc) return rc;
    return check_hip(hipGetLastError(), "k_query launch");
}

int set_query_blocks_per_cu(int v) {
    g_query_blocks_per_cu = v;
    return NIF_OK;
}

int set_query_rays_per_wave(int v) {
    g_query_rays_per_wave = v;
    return NIF_OK;
}

// Times the fused query on the caller's rays for every launch shape of the search space
// (workgroups per CU x rays per wave), keeps the fastest process-wide and reports it.
int autotune_query(const nif_model* m, const nif_grid* g, const nif_rays* r, int64_t n, const nif_hits* out,
                   int32_t precision, int32_t reps, int32_t* best, float* best_ms, hipStream_t st) {
    static const int kBpc[] = {4, 6, 8, 10, 12, 14, 16, 20, 24};
    static const int kRpw[] = {16, 64};
    const int save_bpc = g_query_blocks_per_cu, save_rpw = g_query_rays_per_wave;
    hipEvent_t e0, e1;
    int rc = check_hip(hipEventCreate(&e0), "event");
    if (rc) return rc;
    if ((rc = check_hip(hipEventCreate(&e1), "event"))) { (void)hipEventDestroy(e0); return rc; }
    float best_t = INFINITY;
    int bb = save_bpc, br = save_rpw;
    for (int rpw : kRpw) {
        for (int bpc : kBpc) {
            g_query_blocks_per_cu = bpc;
            g_query_rays_per_wave = rpw;
            if ((rc = query_launch(m, g, r, n, out, 0, precision, nullptr, st))) break;    // warm-up
            if ((rc = check_hip(hipEventRecord(e0, st), "event record"))) break;
            for (int i = 0; i < reps && !rc; ++i) rc = query_launch(m, g, r, n, out, 0, precision, nullptr, st);
            if (rc) break;
            if ((rc = check_hip(hipEventRecord(e1, st), "event record"))) break;
            if ((rc = check_hip(hipEventSynchronize(e1), "event sync"))) break;
            float ms = 0.f;
            if ((rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed"))) break;
            ms /= (float)reps;
            if (ms < best_t) { best_t = ms; bb = bpc; br = rpw; }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_query_blocks_per_cu = rc ? save_bpc : bb;
    g_query_rays_per_wave = rc ? save_rpw : br;
    if (rc) return rc;
    best[0] = bb;
    best[1] = br;
    if (best_ms) *best_ms = best_t;
    return NIF_OK;
}

int encode_launch(const nif_model* m, const float* x, int64_t n, float* out, hipStream_t st) {
    if (n == 0) return NIF_OK;
    const NetParams np = make_net_params(m, NIF_PREC_FP32);
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)device_cus() * 16);
    hipLaunchKernelGGL(k_encode, dim3((unsigned)blocks), dim3(256), 0, st, np.enc, x, n, out);
    return check_hip(hipGetLastError(), "k_encode launch");
}

template <int HW, int PREC>
static void launch_forward(const NetParams& np, const float* x0, const float* x1, int64_t B, int64_t ld, float* heads,
                           float* acts, float* enc, hipStream_t st) {
    // small launches (up to 2^17 pairs) take 16 pairs per wave so that they still fill the chip
    const bool gamma = np.gamma_F >= 0, enc_only = heads == nullptr, small = B <= (1 << 17);
    const int64_t tiles = enc_only || small || np.enc.Fd == 3 ? (B + 15) / 16 : (B + 63) / 64;
    const int64_t blocks = std::min<int64_t>((tiles + 3) / 4, (int64_t)device_cus() * 8);
    const dim3 g((unsigned)std::max<int64_t>(blocks, 1)), b(256);
    if (np.enc.Fd == 3) {            // three-feature entries: 16 pairs per wave throughout
        if (enc_only) hipLaunchKernelGGL((k_forward<HW, PREC, false, true, 16, 3>), g, b, 0, st, np, x0, x1, B, ld, heads, acts, enc);
        else hipLaunchKernelGGL((k_forward<HW, PREC, false, false, 16, 3>), g, b, 0, st, np, x0, x1, B, ld, heads, acts, enc);
        return;
    }
    if (gamma && enc_only) hipLaunchKernelGGL((k_forward<HW, PREC, true, true>), g, b, 0, st, np, x0, x1, B, ld, heads, acts, enc);
    else if (gamma && small) hipLaunchKernelGGL((k_forward<HW, PREC, true, false, 16>), g, b, 0, st, np, x0, x1, B, ld, heads, acts, enc);
    else if (gamma) hipLaunchKernelGGL((k_forward<HW, PREC, true>), g, b, 0, st, np, x0, x1, B, ld, heads, acts, enc);
    else if (enc_only) hipLaunchKernelGGL((k_forward<HW, PREC, false, true>), g, b, 0, st, np, x0, x1, B, ld, heads, acts, enc);
    else if (small) hipLaunchKernelGGL((k_forward<HW, PREC, false, false, 16>), g, b, 0, st, np, x0, x1, B, ld, heads, acts, enc);
    else hipLaunchKernelGGL((k_forward<HW, PREC>), g, b, 0, st, np, x0, x1, B, ld, heads, acts, enc);
}

template <int PREC>
static int dispatch_forward(int hw, const NetParams& np, const float* x0, const float* x1, int64_t B, int64_t ld,
                            float* heads, float* acts, float* enc, hipStream_t st) {
    switch (hw) {
        case 16: launch_forward<16, PREC>(np, x0, x1, B, ld, heads, acts, enc, st); break;
        case 32: launch_forward<32, PREC>(np, x0, x1, B, ld, heads, acts, enc, st); break;
        case 64: launch_forward<64, PREC>(np, x0, x1, B, ld, heads, acts, enc, st); break;
        case 128: launch_forward<128, PREC>(np, x0, x1, B, ld, heads, acts, enc, st); break;
        default: return fail(NIF_E_UNSUPPORTED, "hidden_width must be 16, 32, 64 or 128");
    }
    return NIF_OK;
}

static int forward_any(const nif_model* m, const float* x0, const float* x1, int64_t B, int64_t ld, float* heads,
                       int32_t precision, float* acts, float* enc, hipStream_t st) {
    if (B == 0) return NIF_OK;
    const NetParams np = make_net_params(m, precision);
    const int hw = m->desc.hidden_width;
    int rc;
    if (precision == NIF_PREC_FP32) rc = dispatch_forward<P_FP32>(hw, np, x0, x1, B, ld, heads, acts, enc, st);
    else if (precision == NIF_PREC_BF16) rc = dispatch_forward<P_BF16>(hw, np, x0, x1, B, ld, heads, acts, enc, st);
    else rc = dispatch_forward<P_FP16>(hw, np, x0, x1, B, ld, heads, acts, enc, st);
    if (rc) return rc;
    return check_hip(hipGetLastError(), "k_forward launch");
}

int forward_launch(const nif_model* m, const float* x0, const float* x1, int64_t B, float* heads, int32_t precision,
                   float* acts, float* enc, hipStream_t st) {
    if (heads == nullptr) return fail(NIF_E_INVALID_ARG, "forward needs a heads buffer");
    return forward_any(m, x0, x1, B, B, heads, precision, acts, enc, st);
}

int forward_rows_launch(const nif_model* m, const float* x0, const float* x1, int64_t n, int64_t ld, float* heads,
                        int32_t precision, float* acts, float* enc, hipStream_t st) {
    if (heads == nullptr || ld < n) return fail(NIF_E_INVALID_ARG, "forward needs a heads buffer and ld >= n");
    return forward_any(m, x0, x1, n, ld, heads, precision, acts, enc, st);
}

int encode_pairs_launch(const nif_model* m, const float* x0, const float* x1, int64_t n, int64_t ld, int32_t precision,
                        float* enc, hipStream_t st) {
    if (enc == nullptr || ld < n) return fail(NIF_E_INVALID_ARG, "pair encoding needs an output and ld >= n");
    return forward_any(m, x0, x1, n, ld, nullptr, precision, nullptr, enc, st);
}

}  // namespace nif
