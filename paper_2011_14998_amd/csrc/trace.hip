// Ray tracing through the neighbour graph (Section 2.1, Fig. 2) and the
// device-wide scan that turns ray lengths into list offsets.
//
// One lane walks one ray: from the current point it takes the forward neighbour
// (projection on the ray axis strictly beyond the current one) that lies
// closest to the axis, equal distances going to the smaller point id.  The
// geometry is IEEE FP64 in a fixed operation order with FMA contraction off
// (this file is compiled with -ffp-contract=off as well), so every list is
// bit-identical to any other evaluation of the same rule.
//
// Data layout: neighbour records {x, y, z, id} (32 bytes) in CSR order, built
// once per model, so a step reads one record per neighbour instead of an index
// and then a position.  The whole table of a 50k-point Delaunay mesh (~25 MB)
// stays in the L2/Infinity-cache hierarchy; the walk is latency bound.
#include "rt_internal.h"

#pragma clang fp contract(off)

namespace rt {

namespace {

constexpr int TRACE_BLOCK = 256;

__global__ __launch_bounds__(256) void k_build_nbr(const double* __restrict__ pos, int64_t P,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ idx, int64_t E,
                                                    NbrRec* __restrict__ nbr, int32_t* __restrict__ bad) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= E) return;
    int32_t k = idx[e];
    NbrRec r;
    if (k < 0 || k >= P) {
        atomicOr(bad, 1);
        k = 0;
    }
    r.x = pos[3 * (int64_t)k];
    r.y = pos[3 * (int64_t)k + 1];
    r.z = pos[3 * (int64_t)k + 2];
    r.id = k;
    r.pad = 0;
    nbr[e] = r;
}

__global__ __launch_bounds__(256) void k_check_off(const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                                                    int64_t P, int64_t E, int32_t* __restrict__ bad) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    int64_t a = off[p], b = off[p + 1];
    if (a > b || a < 0 || b > E || (p == 0 && a != 0) || (p == P - 1 && b != E)) {
        atomicOr(bad, 2);
        return;
    }
    for (int64_t e = a; e < b; ++e)
        if (idx[e] == p) atomicOr(bad, 4);
}

template <bool WRITE>
__global__ __launch_bounds__(TRACE_BLOCK) void k_trace(const double* __restrict__ pos, const int64_t* __restrict__ off,
                                                        const NbrRec* __restrict__ nbr, int64_t P,
                                                        const int32_t* __restrict__ origins, int64_t n_origins,
                                                        int64_t R, const double* __restrict__ dirs, int per_origin,
                                                        int32_t* __restrict__ lens, const int64_t* __restrict__ ray_off,
                                                        int32_t* __restrict__ ids, double* __restrict__ Zout,
                                                        int64_t capacity, int32_t* __restrict__ err) {
    const int64_t ray = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t two_r = 2 * R;
    if (ray >= n_origins * two_r) return;
    const int64_t oi = ray / two_r;
    const int64_t rr = ray - oi * two_r;
    const int64_t r = rr >> 1;
    const int64_t o = origins ? (int64_t)origins[oi] : oi;
    if (o < 0 || o >= P) {  // invalid origin id: empty ray, error latched
        if (!WRITE) lens[ray] = 0;
        else atomicOr(err, ERRBIT_ORIGIN);
        return;
    }
    const double* dv = dirs + 3 * ((per_origin ? oi * R : 0) + r);
    double dx = dv[0], dy = dv[1], dz = dv[2];
    if (rr & 1) {
        dx = -dx;
        dy = -dy;
        dz = -dz;
    }
    const double ox = pos[3 * o], oy = pos[3 * o + 1], oz = pos[3 * o + 2];
    int64_t base = 0, room = 0;
    if (WRITE) {
        base = ray_off[ray];
        room = ray_off[ray + 1] - base;
        if (base + room > capacity) room = capacity - base;
    }
    int64_t c = o, n = 0;
    double Zc = 0.0;
    for (int64_t step = 0; step < P; ++step) {
        const int64_t e0 = off[c], e1 = off[c + 1];
        int32_t best = -1;
        double bestD = 0.0, bestZ = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            const NbrRec rec = nbr[e];
            const double Rx = rec.x - ox, Ry = rec.y - oy, Rz = rec.z - oz;
            const double Zk = (Rx * dx + Ry * dy) + Rz * dz;
            if (!(Zk > Zc)) continue;
            const double qx = Rx - Zk * dx, qy = Ry - Zk * dy, qz = Rz - Zk * dz;
            const double Dk = (qx * qx + qy * qy) + qz * qz;
            if (best < 0 || Dk < bestD || (Dk == bestD && rec.id < best)) {
                best = rec.id;
                bestD = Dk;
                bestZ = Zk;
            }
        }
        if (best < 0) break;
        if (WRITE) {
            if (n < room) {
                ids[base + n] = best;
                Zout[base + n] = bestZ;
            } else {
                atomicOr(err, ERRBIT_CAPACITY);
                break;
            }
        }
        ++n;
        c = best;
        Zc = bestZ;
    }
    if (!WRITE) lens[ray] = (int32_t)n;
}

// ---------------------------------------------------------------- scan
// Exclusive scan of int32 lengths into int64 offsets, off[n] = total.
// Pass 1: per-tile sums; pass 2: one block scans the tile sums; pass 3: each
// tile scans itself and adds its tile offset.
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int64_t SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < SCAN_BLOCK; d <<= 1) {
        int64_t add = (t >= d) ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    *total = sh[SCAN_BLOCK - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles(const int32_t* __restrict__ in, int64_t n,
                                                            int64_t* __restrict__ tile_sum) {
    __shared__ int64_t sh[SCAN_BLOCK];
    const int64_t t0 = blockIdx.x * SCAN_TILE;
    int64_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = t0 + (int64_t)i * SCAN_BLOCK + threadIdx.x;
        if (k < n) s += in[k];
    }
    int64_t tot;
    block_exclusive_scan(s, sh, &tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_sums(int64_t* __restrict__ tile_sum, int64_t n_tiles,
                                                           int64_t* __restrict__ out, int64_t n) {
    __shared__ int64_t sh[SCAN_BLOCK];
    int64_t carry = 0;
    for (int64_t b = 0; b < n_tiles; b += SCAN_BLOCK) {
        int64_t k = b + threadIdx.x;
        int64_t v = k < n_tiles ? tile_sum[k] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan(v, sh, &tot);
        if (k < n_tiles) tile_sum[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                            const int64_t* __restrict__ tile_off,
                                                            int64_t* __restrict__ out) {
    __shared__ int64_t sh[SCAN_BLOCK];
    // each thread owns SCAN_ITEMS consecutive elements of the tile
    const int64_t t0 = blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = t0 + i;
        v[i] = k < n ? in[k] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t run = tile_off[blockIdx.x] + block_exclusive_scan(s, sh, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = t0 + i;
        if (k < n) out[k] = run;
        run += v[i];
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_build_nbr(const rt_model* m, int32_t* bad, hipStream_t s) {
    if (m->E > 0)
        hipLaunchKernelGGL(k_build_nbr, dim3(blocks_for(m->E, 256)), dim3(256), 0, s, m->pos, m->P, m->off, m->idx,
                           m->E, m->nbr, bad);
    hipLaunchKernelGGL(k_check_off, dim3(blocks_for(m->P, 256)), dim3(256), 0, s, m->off, m->idx, m->P, m->E, bad);
    return hipGetLastError();
}

hipError_t launch_trace_count(const rt_model* m, const int32_t* origins, int64_t n_origins, int64_t R,
                              const double* dirs, int per_origin, int32_t* lens, hipStream_t s) {
    int64_t n = n_origins * 2 * R;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_trace<false>, dim3(blocks_for(n, TRACE_BLOCK)), dim3(TRACE_BLOCK), 0, s, m->pos, m->off,
                       m->nbr, m->P, origins, n_origins, R, dirs, per_origin, lens, nullptr, nullptr, nullptr,
                       (int64_t)0, nullptr);
    return hipGetLastError();
}

hipError_t launch_trace_write(const rt_model* m, const int32_t* origins, int64_t n_origins, int64_t R,
                              const double* dirs, int per_origin, const int64_t* ray_off, int32_t* ids,
                              double* Z, int64_t capacity, hipStream_t s) {
    int64_t n = n_origins * 2 * R;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_trace<true>, dim3(blocks_for(n, TRACE_BLOCK)), dim3(TRACE_BLOCK), 0, s, m->pos, m->off,
                       m->nbr, m->P, origins, n_origins, R, dirs, per_origin, nullptr, ray_off, ids, Z, capacity,
                       error_word());
    return hipGetLastError();
}

size_t scan_workspace(int64_t n) {
    int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    return (size_t)(tiles > 0 ? tiles : 1) * sizeof(int64_t);
}

hipError_t launch_scan(const int32_t* lens, int64_t n, int64_t* off, void* ws, hipStream_t s) {
    int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    int64_t* tile_sum = (int64_t*)ws;
    if (tiles > 0)
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, lens, n, tile_sum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_BLOCK), 0, s, tile_sum, tiles, off, n);
    if (tiles > 0)
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, lens, n, tile_sum, off);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace rt
