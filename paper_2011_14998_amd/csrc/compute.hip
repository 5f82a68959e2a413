// The whole path in one call, and many models in one launch.
//
// rt_compute_J: trace (count, scan, write), sweep and J for a list of origins
// inside the caller's workspace.  The origins are put in Morton order of their
// positions and cut into consecutive chunks whose ray lists fit the space left
// after the fixed per-origin parts: a window of origins is counted, and the
// chunk is the longest prefix of the window whose lists fit (read from the
// scanned offsets at origin boundaries); the counts of the rest of the window
// carry over to the next chunk, so every origin is counted once.  Rays and
// sweep items of a chunk run direction by direction over that order, and the
// J rows are scattered back to the caller's list order.
//
// rt_batch: a disjoint union of many models built on the device, traced and
// solved by one plan; table gather, the plan's step and the scatter of J to
// each model are one HIP graph.  Model k's points take the union ids base_k ..
// base_k + P_k - 1 in the Morton order of that model's positions, so points that
// are near in space are near in the neighbour records and the tables the walk
// and the sweep read (direction-major over that same order).  Positions are not
// moved and each union row keeps the order of the model's own neighbour ids, so
// every ray and every result is the one the model alone gives.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rt_internal.h"

namespace rt {

namespace {

inline size_t al(size_t v) { return (v + 255) / 256 * 256; }
inline unsigned blocks_of(int64_t n, int b) { return capped_blocks((n + b - 1) / b); }

__global__ void k_iota(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

// dst[k] = src[perm[k]], or perm[k] itself when src is NULL (origins 0..n-1)
__global__ void k_permute_ids(const int32_t* __restrict__ src, const int32_t* __restrict__ perm, int64_t n,
                              int32_t* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src ? src[perm[i]] : perm[i];
}

// rows of `width` values: dst[perm[k]][:] = src[k][:]
template <typename T>
__global__ void k_scatter_rows(const T* __restrict__ src, const int32_t* __restrict__ perm, int64_t n, int64_t width,
                               T* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * width;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = i / width, c = i - k * width;
        dst[(int64_t)perm[k] * width + c] = src[i];
    }
}

__global__ void k_shift_i64(const int64_t* __restrict__ src, int64_t n, int64_t shift, int64_t* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] + shift;
}

__global__ void k_shift_i32(const int32_t* __restrict__ src, int64_t n, int32_t shift, int32_t* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] + shift;
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

// out[k] = off[k * stride] for k <= n (list offsets at origin boundaries)
__global__ void k_gather_bounds(const int64_t* __restrict__ off, int64_t stride, int64_t n, int64_t* __restrict__ out) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= n; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = off[k * stride];
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int64_t n, int32_t* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Union point u is point perm[u] of the models' concatenation (model after model, ids
// shifted by base_k): its position, velocity and degree.
__global__ void k_union_points(const int32_t* __restrict__ perm, int64_t P, const double* __restrict__ pos_c,
                               const float* __restrict__ vel_c, const int64_t* __restrict__ off_c,
                               double* __restrict__ pos, float* __restrict__ vel, int32_t* __restrict__ deg) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < P; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = perm[u];
        for (int i = 0; i < 3; ++i) pos[3 * u + i] = pos_c[3 * c + i];
        if (vel) for (int i = 0; i < 3; ++i) vel[3 * u + i] = vel_c[3 * c + i];
        deg[u] = (int32_t)(off_c[c + 1] - off_c[c]);
    }
}

// Union row u: the neighbours of concatenated point perm[u], renamed to union ids.
__global__ void k_union_rows(const int32_t* __restrict__ perm, const int32_t* __restrict__ uid, int64_t P,
                             const int64_t* __restrict__ off_c, const int32_t* __restrict__ idx_c,
                             const int64_t* __restrict__ off, int32_t* __restrict__ idx) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < P; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = perm[u], a = off_c[c], n = off_c[c + 1] - a, d = off[u];
        for (int64_t j = 0; j < n; ++j) idx[d + j] = uid[idx_c[a + j]];
    }
}

// One model of a batch: its tables, its J and where its points start in the union.
struct BatchSeg {
    const void* chi;
    const void* eta;
    void* J;
    int64_t ld;
    int64_t P;
    int64_t base;
};

// Union tables [P_total][F] from the models' [P_k][ld_k] tables; model k = blockIdx.y, union
// row base_k + r holds the model's row lrow[base_k + r].
template <typename T>
__global__ __launch_bounds__(256) void k_batch_gather(const BatchSeg* __restrict__ segs,
                                                      const int32_t* __restrict__ lrow, int64_t F,
                                                      T* __restrict__ chi_u, T* __restrict__ eta_u) {
    const BatchSeg g = segs[blockIdx.y];
    const T* __restrict__ c = (const T*)g.chi;
    const T* __restrict__ e = (const T*)g.eta;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.P * F; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / F, f = i - r * F, src = lrow[g.base + r];
        chi_u[(g.base + r) * F + f] = c[src * g.ld + f];
        eta_u[(g.base + r) * F + f] = e[src * g.ld + f];
    }
}

// Each model's J [P_k][F] from the union's J rows.
template <typename T>
__global__ __launch_bounds__(256) void k_batch_scatter(const BatchSeg* __restrict__ segs,
                                                       const int32_t* __restrict__ lrow, int64_t F,
                                                       const T* __restrict__ J_u) {
    const BatchSeg g = segs[blockIdx.y];
    T* __restrict__ J = (T*)g.J;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.P * F; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / F, f = i - r * F;
        J[lrow[g.base + r] * F + f] = J_u[(g.base + r) * F + f];
    }
}

// Bytes of the per-chunk parts of the workspace for windows and chunks of up
// to c origins (everything but the ray lists), and where each part starts:
// two buffers of ray lengths (the window's, and the carried-over rest), the
// offsets and their scan space, the origin-boundary offsets, per-pair u, the
// chunk's J rows and the bins.
struct ChunkParts {
    size_t identity, lens, lens2, off, bnd, scan, u, Jc, bins, total;
};

ChunkParts chunk_parts(int64_t c, int64_t R, int64_t F, size_t es, bool permute, bool binned) {
    ChunkParts p;
    const int64_t rays = c * 2 * R;
    p.identity = 0;
    p.lens = p.identity + al(sizeof(int32_t) * (size_t)std::max<int64_t>(c, 1));
    p.lens2 = p.lens + al(sizeof(int32_t) * (size_t)std::max<int64_t>(rays, 1));
    p.off = p.lens2 + al(sizeof(int32_t) * (size_t)std::max<int64_t>(rays, 1));
    p.bnd = p.off + al(sizeof(int64_t) * (size_t)(rays + 1));
    p.scan = p.bnd + al(sizeof(int64_t) * (size_t)(c + 1));
    p.u = p.scan + al(scan_workspace(rays));
    p.Jc = p.u + al(es * (size_t)std::max<int64_t>(c * R * F, 1));
    p.bins = p.Jc + (permute ? al(es * (size_t)std::max<int64_t>(c * F, 1)) : 0);
    const int64_t items = c * R * ((F + 63) / 64);
    p.total = p.bins + (binned ? 256 + al(bin_workspace(items, 128)) : 0);
    return p;
}

size_t global_parts(int64_t n, bool permute, bool need_ids) {
    // permutation (list positions in chunk order) and the permuted origin ids
    return (permute ? 2 * al(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1)) : 0) +
           (!permute && need_ids ? al(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1)) : 0);
}

int64_t grid_F(const rt_freq_grid* g) {
    int64_t F = 0;
    for (int b = 0; b < g->n_blocks && g->len; ++b) F += g->len[b];
    return F;
}

}  // namespace

size_t compute_ws_fixed(int64_t n_origins, int64_t R, int64_t F, const rt_solve_opts& o) {
    const size_t es = o.precision == RT_F64 ? 8 : 4;
    return global_parts(n_origins, true, true) +
           chunk_parts(n_origins, R, F, es, true, o.schedule == RT_SCHED_BINNED).total;
}

}  // namespace rt

using namespace rt;

extern "C" rt_status rt_compute_J_workspace(const rt_dirset* set, int64_t n_origins, int64_t F,
                                            const rt_solve_opts* opts, double mean_entries, size_t* bytes) {
    if (!set || !bytes || n_origins < 0 || F <= 0) return fail(RT_ERR_ARG, "rt_compute_J_workspace: bad arguments");
    const rt_solve_opts o = opts ? *opts : default_solve_opts();
    const bool permute = set->n_origins == 0;
    const size_t es = o.precision == RT_F64 ? 8 : 4;
    const double L = mean_entries > 0.0 ? mean_entries : 64.0;
    const double entries = (double)n_origins * 2.0 * (double)set->R * L;
    *bytes = global_parts(n_origins, permute, true) +
             chunk_parts(n_origins, set->R, F, es, permute, o.schedule == RT_SCHED_BINNED).total +
             al((size_t)(1.1 * 4.0 * entries)) + al((size_t)(1.1 * 8.0 * entries)) + 2048;
    return RT_OK;
}

extern "C" rt_status rt_compute_J(const rt_model* m, const rt_dirset* set_, const int32_t* origins, int64_t n,
                                  const void* chi, const void* eta, int32_t dtype, int64_t ld,
                                  const rt_freq_grid* grid, const double* I_bc, void* J, void* u_out,
                                  const rt_solve_opts* opts, void* ws, size_t ws_bytes, void* stream) {
    rt_dirset* set = const_cast<rt_dirset*>(set_);
    const rt_solve_opts o = opts ? *opts : default_solve_opts();
    if (o.schedule < RT_SCHED_DIRECT || o.schedule > RT_SCHED_SPATIAL)
        return fail(RT_ERR_ARG, "rt_compute_J: bad schedule");
    if (o.trace_lanes != 0 && o.trace_lanes != 4 && o.trace_lanes != 8 && o.trace_lanes != 16)
        return fail(RT_ERR_ARG, "rt_compute_J: trace_lanes must be 4, 8 or 16");
    if (n < 0) return fail(RT_ERR_ARG, "rt_compute_J: negative origin count");
    SolveLaunch base;
    rt_status st = fill_solve_launch(m, set, origins, n, nullptr, nullptr, nullptr, chi, eta, dtype, ld, grid, I_bc,
                                     J, o, base);
    if (st) return st;
    if (n == 0) return RT_OK;
    if (!ws) return fail(RT_ERR_CAPACITY, "rt_compute_J: no workspace");
    hipStream_t s = (hipStream_t)stream;
    const int64_t R = set->R, F = base.F;
    const int per = set->n_origins > 0;
    const bool permute = !per;
    const bool binned = o.schedule == RT_SCHED_BINNED;
    const size_t es = o.precision == RT_F64 ? 8 : 4;
    const int nfc = (int)((F + 63) / 64);
    // global parts: the chunk order and the origin ids in that order
    char* wp = (char*)ws;
    const size_t G = global_parts(n, permute, origins == nullptr);
    if (ws_bytes < G) return fail(RT_ERR_CAPACITY, "rt_compute_J: workspace too small");
    int32_t* perm = nullptr;
    const int32_t* ids_all = origins;
    std::vector<int32_t> order;
    if (permute) {
        perm = (int32_t*)wp;
        int32_t* pids = (int32_t*)(wp + al(sizeof(int32_t) * (size_t)n));
        RT_HIP(morton_order(m, origins, n, s, order));
        RT_HIP(hipMemcpyAsync(perm, order.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_permute_ids, dim3(blocks_of(n, 256)), dim3(256), 0, s, origins, perm, n, pids);
        RT_HIP(hipGetLastError());
        ids_all = pids;
    } else if (!origins) {
        int32_t* iota = (int32_t*)wp;
        hipLaunchKernelGGL(k_iota, dim3(blocks_of(n, 256)), dim3(256), 0, s, iota, n);
        RT_HIP(hipGetLastError());
        ids_all = iota;
    }
    char* cw = wp + G;
    const size_t W = ws_bytes - G;
    // window size: the per-chunk parts for w origins plus the lists of 0.8 w origins at a
    // mean of 64 entries per ray fit the space (a window longer than its chunk keeps the
    // rest of its counts for the next one)
    auto fits = [&](int64_t w) {
        const ChunkParts cp = chunk_parts(w, R, F, es, permute, binned);
        const double lists = 0.8 * (double)w * 2.0 * (double)R * 64.0 * 12.0 + 1024.0;
        return (double)cp.total + lists <= (double)W;
    };
    int64_t lo = 0, hi = std::min<int64_t>(n, MAX_SOLVE_ITEMS / (R * nfc));
    while (lo < hi) {  // largest window that fits
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (fits(mid)) lo = mid;
        else hi = mid - 1;
    }
    int64_t wmax = std::max<int64_t>(lo, 1);
    ChunkParts cp = chunk_parts(wmax, R, F, es, permute, binned);
    while (cp.total + 1024 > W && wmax > 1) cp = chunk_parts(wmax /= 2, R, F, es, permute, binned);
    if (cp.total + 1024 > W) return fail(RT_ERR_CAPACITY, "rt_compute_J: workspace below the fixed part for one origin");
    const int64_t cap = (int64_t)((W - cp.total - 512) / 12);
    int32_t* identity = (int32_t*)(cw + cp.identity);
    int32_t* lens = (int32_t*)(cw + cp.lens);
    int32_t* lens_rest = (int32_t*)(cw + cp.lens2);
    int64_t* off = (int64_t*)(cw + cp.off);
    int64_t* bnd = (int64_t*)(cw + cp.bnd);
    void* scan_ws = cw + cp.scan;
    char* u_c = cw + cp.u;
    char* J_c = cw + cp.Jc;
    char* lists = cw + cp.total;
    int32_t* ids = (int32_t*)lists;
    double* Z = (double*)(lists + al(sizeof(int32_t) * (size_t)std::max<int64_t>(cap, 1)));
    hipLaunchKernelGGL(k_iota, dim3(blocks_of(wmax, 256)), dim3(256), 0, s, identity, wmax);
    RT_HIP(hipGetLastError());
    std::vector<int64_t> hb;
    int64_t c0 = 0, have = 0;  // origins [c0, c0 + have) are counted, their lengths in lens
    while (c0 < n) {
        const int64_t want = std::min(n - c0, wmax);
        if (have < want) {  // count the window's new origins
            const int64_t a0 = c0 + have, extra = want - have;
            RT_HIP(launch_trace_count(m, ids_all + a0, extra, R, set->d_dirs() + (per ? 3 * R * a0 : 0), per,
                                      lens + have * 2 * R, s, identity, o.trace_lanes));
            have = want;
        }
        RT_HIP(launch_scan(lens, have * 2 * R, off, scan_ws, s));
        hipLaunchKernelGGL(k_gather_bounds, dim3(blocks_of(have + 1, 256)), dim3(256), 0, s, off, 2 * R, have, bnd);
        RT_HIP(hipGetLastError());
        hb.resize((size_t)(have + 1));
        RT_HIP(hipMemcpyAsync(hb.data(), bnd, sizeof(int64_t) * (size_t)(have + 1), hipMemcpyDeviceToHost, s));
        RT_HIP(hipStreamSynchronize(s));
        // the chunk: the longest prefix of the window whose lists fit
        const int64_t c = (int64_t)(std::upper_bound(hb.begin(), hb.end(), cap) - hb.begin()) - 1;
        if (c < 1) return fail(RT_ERR_CAPACITY, "rt_compute_J: one origin's rays do not fit the workspace");
        const int64_t total = hb[(size_t)c];
        const int32_t* org_c = ids_all + c0;
        const double* dirs_c = set->d_dirs() + (per ? 3 * R * c0 : 0);
        const double* w2_c = set->d_w2() + (per ? R * c0 : 0);
        RT_HIP(launch_trace_write(m, org_c, c, R, dirs_c, per, off, ids, Z, total, s, identity, o.trace_lanes));
        SolveLaunch a = base;
        a.origins = org_c;
        a.n_origins = c;
        a.dirs = dirs_c;
        a.w2 = w2_c;
        a.ray_off = off;
        a.ray_ids = ids;
        a.ray_Z = Z;
        a.u = (!permute && u_out) ? (void*)((char*)u_out + es * (size_t)(c0 * R * F)) : (void*)u_c;
        a.J = permute ? (void*)J_c : (void*)((char*)J + es * (size_t)(c0 * F));
        a.schedule = binned ? RT_SCHED_BINNED : RT_SCHED_DIRECT;
        a.order = o.schedule == RT_SCHED_DIRECT ? nullptr : identity;
        a.items = nullptr;
        a.queue = nullptr;
        if (binned) {
            a.queue = (int32_t*)(cw + cp.bins);
            int32_t* items = nullptr;
            RT_HIP(launch_bin(a, cw + cp.bins + 256, &items, s));
            a.items = items;
            RT_HIP(launch_fill_i32(a.queue, 1, 0, s));
        }
        RT_HIP(launch_solve(a, o.precision, s));
        RT_HIP(launch_reduce(a, o.precision, s));
        if (permute) {
            if (o.precision == RT_F64) {
                hipLaunchKernelGGL(k_scatter_rows<double>, dim3(blocks_of(c * F, 256)), dim3(256), 0, s,
                                   (const double*)J_c, perm + c0, c, F, (double*)J);
                if (u_out)
                    hipLaunchKernelGGL(k_scatter_rows<double>, dim3(blocks_of(c * R * F, 256)), dim3(256), 0, s,
                                       (const double*)u_c, perm + c0, c, R * F, (double*)u_out);
            } else {
                hipLaunchKernelGGL(k_scatter_rows<float>, dim3(blocks_of(c * F, 256)), dim3(256), 0, s,
                                   (const float*)J_c, perm + c0, c, F, (float*)J);
                if (u_out)
                    hipLaunchKernelGGL(k_scatter_rows<float>, dim3(blocks_of(c * R * F, 256)), dim3(256), 0, s,
                                       (const float*)u_c, perm + c0, c, R * F, (float*)u_out);
            }
            RT_HIP(hipGetLastError());
        }
        // the window's uncut origins keep their counts
        const int64_t rest = have - c;
        if (rest > 0) {
            hipLaunchKernelGGL(k_copy_i32, dim3(blocks_of(rest * 2 * R, 256)), dim3(256), 0, s, lens + c * 2 * R,
                               rest * 2 * R, lens_rest);
            RT_HIP(hipGetLastError());
            std::swap(lens, lens_rest);
        }
        have = rest;
        c0 += c;
    }
    return RT_OK;
}

// ------------------------------------------------------------------ many models

struct rt_batch {
    int n = 0;
    std::vector<int64_t> P, base_p, E, base_e;
    std::vector<const void*> chi, eta;
    std::vector<int64_t> ld;
    std::vector<void*> J;
    int32_t dtype = RT_F32;
    int64_t F = 0, P_tot = 0, E_tot = 0;
    double* pos = nullptr;
    int64_t* off = nullptr;
    int32_t* idx = nullptr;
    float* vel = nullptr;
    void* chi_u = nullptr;
    void* eta_u = nullptr;
    void* J_u = nullptr;
    BatchSeg* segs = nullptr;  // device [n]
    int32_t* lrow = nullptr;   // device [P_tot]: the model row of each union point
    int32_t* uid = nullptr;    // device [P_tot]: the union id of point base_k + i of model k
    int64_t max_P = 0;
    rt_model* uni = nullptr;
    rt_plan* plan = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t captured = -1;  // plan version the graph holds
};

static void batch_free(rt_batch* b) {
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->plan) rt_plan_destroy(b->plan);
    if (b->uni) rt_model_destroy(b->uni);
    for (void* q : {(void*)b->pos, (void*)b->off, (void*)b->idx, (void*)b->vel, b->chi_u, b->eta_u, b->J_u,
                    (void*)b->segs, (void*)b->lrow, (void*)b->uid})
        if (q) (void)hipFree(q);
    delete b;
}

// The models' tables into the union.
static hipError_t batch_gather(rt_batch* b, hipStream_t s) {
    const dim3 grid(std::min<unsigned>(2048, blocks_of(b->max_P * b->F, 256)), (unsigned)b->n);
    if (b->dtype == RT_F64)
        hipLaunchKernelGGL(k_batch_gather<double>, grid, dim3(256), 0, s, b->segs, b->lrow, b->F, (double*)b->chi_u,
                           (double*)b->eta_u);
    else
        hipLaunchKernelGGL(k_batch_gather<float>, grid, dim3(256), 0, s, b->segs, b->lrow, b->F, (float*)b->chi_u,
                           (float*)b->eta_u);
    return hipGetLastError();
}

// Gather the tables into the union, run the plan's step, scatter J to the models.
static hipError_t batch_enqueue(rt_batch* b, hipStream_t s) {
    const dim3 grid(std::min<unsigned>(2048, blocks_of(b->max_P * b->F, 256)), (unsigned)b->n);
    hipError_t e = batch_gather(b, s);
    if (e == hipSuccess) e = plan_enqueue_step(b->plan, s);
    if (e != hipSuccess) return e;
    if (b->dtype == RT_F64)
        hipLaunchKernelGGL(k_batch_scatter<double>, grid, dim3(256), 0, s, b->segs, b->lrow, b->F,
                           (const double*)b->J_u);
    else
        hipLaunchKernelGGL(k_batch_scatter<float>, grid, dim3(256), 0, s, b->segs, b->lrow, b->F,
                           (const float*)b->J_u);
    return hipGetLastError();
}

static rt_status batch_capture(rt_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = batch_enqueue(b, cap);
        e = hipStreamEndCapture(cap, &b->graph);
        if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return hip_fail(e, "rt_batch: graph capture");
    b->captured = plan_version(b->plan);
    return RT_OK;
}

extern "C" rt_status rt_batch_create(int32_t n_models, const rt_model* const* models, const rt_dirset* set_,
                                     const void* const* chi, const void* const* eta, int32_t dtype, const int64_t* ld,
                                     const rt_freq_grid* grid, const double* I_bc, void* const* J,
                                     const rt_solve_opts* opts, void* stream, rt_batch** out) {
    if (!out) return fail(RT_ERR_ARG, "rt_batch_create: NULL output");
    *out = nullptr;
    rt_dirset* set = const_cast<rt_dirset*>(set_);
    if (n_models <= 0 || !models || !set || !chi || !eta || !ld || !grid || !I_bc || !J)
        return fail(RT_ERR_ARG, "rt_batch_create: NULL argument or no models");
    if (set->n_origins > 0) return fail(RT_ERR_ARG, "rt_batch_create: the direction set must be shared (uniform)");
    if (dtype != RT_F32 && dtype != RT_F64) return fail(RT_ERR_ARG, "rt_batch_create: dtype must be RT_F32 or RT_F64");
    const int64_t F = grid_F(grid);
    if (F <= 0) return fail(RT_ERR_ARG, "rt_batch_create: empty frequency grid");
    int dev = 0;
    RT_HIP(hipGetDevice(&dev));
    hipStream_t s = (hipStream_t)stream;
    auto* b = new rt_batch();
    b->n = n_models;
    b->dtype = dtype;
    b->F = F;
    bool moving = false;
    for (int k = 0; k < n_models; ++k) {
        const rt_model* m = models[k];
        if (!m || !chi[k] || !eta[k] || !J[k] || ld[k] < F) {
            delete b;
            return fail(RT_ERR_ARG, "rt_batch_create: NULL model, table or J, or ld < F");
        }
        if (m->device != dev) {
            delete b;
            return fail(RT_ERR_ARG, "rt_batch_create: a model lives on another device");
        }
        b->P.push_back(m->P);
        b->E.push_back(m->E);
        b->base_p.push_back(b->P_tot);
        b->base_e.push_back(b->E_tot);
        b->P_tot += m->P;
        b->E_tot += m->E;
        b->chi.push_back(chi[k]);
        b->eta.push_back(eta[k]);
        b->ld.push_back(ld[k]);
        b->J.push_back(J[k]);
        moving = moving || m->vel != nullptr;
    }
    b->base_p.push_back(b->P_tot);
    if (b->P_tot > INT32_MAX || b->E_tot > INT32_MAX) {
        delete b;
        return fail(RT_ERR_UNSUPPORTED, "rt_batch_create: more than 2^31-1 points or entries in the union");
    }
    const size_t es = dtype == RT_F64 ? 8 : 4;
    hipError_t e = hipMalloc((void**)&b->pos, sizeof(double) * 3 * (size_t)b->P_tot);
    if (e == hipSuccess) e = hipMalloc((void**)&b->off, sizeof(int64_t) * (size_t)(b->P_tot + 1));
    if (e == hipSuccess) e = hipMalloc((void**)&b->idx, sizeof(int32_t) * (size_t)std::max<int64_t>(b->E_tot, 1));
    if (e == hipSuccess && moving) e = hipMalloc((void**)&b->vel, sizeof(float) * 3 * (size_t)b->P_tot);
    if (e == hipSuccess) e = hipMalloc(&b->chi_u, es * (size_t)(b->P_tot * F));
    if (e == hipSuccess) e = hipMalloc(&b->eta_u, es * (size_t)(b->P_tot * F));
    if (e == hipSuccess) e = hipMalloc(&b->J_u, es * (size_t)(b->P_tot * F));
    if (e == hipSuccess) e = hipMalloc((void**)&b->segs, sizeof(BatchSeg) * (size_t)n_models);
    if (e == hipSuccess) {
        std::vector<BatchSeg> hs((size_t)n_models);
        for (int k = 0; k < n_models; ++k) {
            hs[(size_t)k] = BatchSeg{chi[k], eta[k], J[k], ld[k], b->P[(size_t)k], b->base_p[(size_t)k]};
            b->max_P = std::max(b->max_P, b->P[(size_t)k]);
        }
        e = hipMemcpy(b->segs, hs.data(), sizeof(BatchSeg) * hs.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, s, b->off);
    for (int k = 0; k < n_models && e == hipSuccess; ++k) {
        const rt_model* m = models[k];
        const int64_t bp = b->base_p[(size_t)k], be = b->base_e[(size_t)k];
        e = hipMemcpyAsync(b->pos + 3 * bp, m->pos, sizeof(double) * 3 * (size_t)m->P, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            hipLaunchKernelGGL(k_shift_i64, dim3(blocks_of(m->P, 256)), dim3(256), 0, s, m->off + 1, m->P, be,
                               b->off + bp + 1);
        if (e == hipSuccess && m->E > 0)
            hipLaunchKernelGGL(k_shift_i32, dim3(blocks_of(m->E, 256)), dim3(256), 0, s, m->idx, m->E, (int32_t)bp,
                               b->idx + be);
        if (e == hipSuccess && moving) {
            if (m->vel)
                e = hipMemcpyAsync(b->vel + 3 * bp, m->vel, sizeof(float) * 3 * (size_t)m->P, hipMemcpyDeviceToDevice,
                                   s);
            else
                hipLaunchKernelGGL(k_fill_f32, dim3(blocks_of(3 * m->P, 256)), dim3(256), 0, s, b->vel + 3 * bp,
                                   3 * m->P, 0.f);
        }
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e != hipSuccess) {
        rt_status st = hip_fail(e, "rt_batch_create");
        batch_free(b);
        return st;
    }
    // The concatenation is renumbered: union point u = concatenated point perm[u], each model's
    // points in the Morton order of its own positions.
    const int64_t Pt = b->P_tot;
    std::vector<int32_t> perm, uid_h((size_t)Pt), lrow_h((size_t)Pt);
    std::vector<double> hpos_seg((size_t)(3 * Pt));  // concatenation order: model k at base_k ..
    e = hipMemcpyAsync(hpos_seg.data(), b->pos, sizeof(double) * hpos_seg.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) morton_order_host(hpos_seg.data(), Pt, nullptr, Pt, perm, b->base_p.data(), n_models);
    if (e == hipSuccess)
        for (int k = 0; k < n_models; ++k)
            for (int64_t u = b->base_p[(size_t)k]; u < b->base_p[(size_t)k + 1]; ++u) {
                const int32_t c = perm[(size_t)u];
                uid_h[(size_t)c] = (int32_t)u;
                lrow_h[(size_t)u] = (int32_t)(c - b->base_p[(size_t)k]);
            }
    double* pos_u = nullptr;
    int64_t* off_u = nullptr;
    int32_t *idx_u = nullptr, *perm_d = nullptr, *deg = nullptr;
    float* vel_u = nullptr;
    void* scan_ws = nullptr;
    if (e == hipSuccess) e = hipMalloc((void**)&pos_u, sizeof(double) * 3 * (size_t)Pt);
    if (e == hipSuccess) e = hipMalloc((void**)&off_u, sizeof(int64_t) * (size_t)(Pt + 1));
    if (e == hipSuccess) e = hipMalloc((void**)&idx_u, sizeof(int32_t) * (size_t)std::max<int64_t>(b->E_tot, 1));
    if (e == hipSuccess && moving) e = hipMalloc((void**)&vel_u, sizeof(float) * 3 * (size_t)Pt);
    if (e == hipSuccess) e = hipMalloc((void**)&perm_d, sizeof(int32_t) * (size_t)Pt);
    if (e == hipSuccess) e = hipMalloc((void**)&deg, sizeof(int32_t) * (size_t)Pt);
    if (e == hipSuccess) e = hipMalloc(&scan_ws, std::max<size_t>(scan_workspace(Pt), 1));
    if (e == hipSuccess) e = hipMalloc((void**)&b->uid, sizeof(int32_t) * (size_t)Pt);
    if (e == hipSuccess) e = hipMalloc((void**)&b->lrow, sizeof(int32_t) * (size_t)Pt);
    if (e == hipSuccess) e = hipMemcpyAsync(perm_d, perm.data(), sizeof(int32_t) * (size_t)Pt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->uid, uid_h.data(), sizeof(int32_t) * (size_t)Pt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->lrow, lrow_h.data(), sizeof(int32_t) * (size_t)Pt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_union_points, dim3(blocks_of(Pt, 256)), dim3(256), 0, s, perm_d, Pt, b->pos, b->vel, b->off,
                           pos_u, vel_u, deg);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_scan(deg, Pt, off_u, scan_ws, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_union_rows, dim3(blocks_of(Pt, 256)), dim3(256), 0, s, perm_d, b->uid, Pt, b->off, b->idx,
                           off_u, idx_u);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // the renumbered arrays replace the concatenation
    std::swap(b->pos, pos_u);
    std::swap(b->off, off_u);
    std::swap(b->idx, idx_u);
    if (moving) std::swap(b->vel, vel_u);
    for (void* q : {(void*)pos_u, (void*)off_u, (void*)idx_u, (void*)vel_u, (void*)deg, scan_ws})
        if (q) (void)hipFree(q);
    if (e != hipSuccess) {
        if (perm_d) (void)hipFree(perm_d);
        rt_status st = hip_fail(e, "rt_batch_create: union order");
        batch_free(b);
        return st;
    }
    // rows in the order of the concatenation's ids (the models' own order), as each model alone has them
    rt_status st = model_create(b->pos, Pt, b->off, b->idx, b->E_tot, b->vel, perm_d, false, s, &b->uni);
    (void)hipFree(perm_d);
    if (st) {
        batch_free(b);
        return st;
    }
    // origins: every point in union order (each model's points in Morton order already); the
    // sweep's per-pair orders keep the models apart, each in its own bounding sphere
    std::vector<int32_t> order((size_t)Pt);
    for (int64_t u = 0; u < Pt; ++u) order[(size_t)u] = (int32_t)u;
    std::vector<OrderSeg> segs((size_t)n_models);
    for (int k = 0; k < n_models; ++k) {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t q = b->base_p[(size_t)k]; q < b->base_p[(size_t)k + 1]; ++q)
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::min(lo[c], hpos_seg[(size_t)(3 * q + c)]);
                hi[c] = std::max(hi[c], hpos_seg[(size_t)(3 * q + c)]);
            }
        OrderSeg& g = segs[(size_t)k];
        g.end = b->base_p[(size_t)k + 1];
        double r2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            g.c[c] = 0.5 * (lo[c] + hi[c]);
            r2 += 0.25 * (hi[c] - lo[c]) * (hi[c] - lo[c]);
        }
        g.rho = std::sqrt(r2);
    }
    // the union's tables hold the models' values from the start, so that the inner plan can be run,
    // profiled or tuned on its own (rt_batch_plan) before the first rt_batch_run
    e = batch_gather(b, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        st = hip_fail(e, "rt_batch_create: table gather");
        batch_free(b);
        return st;
    }
    st = plan_create_ordered(b->uni, set, nullptr, b->P_tot, b->chi_u, b->eta_u, dtype, F, grid, I_bc, b->J_u, opts,
                             s, &order, &b->plan, &segs);
    if (!st) st = batch_capture(b);
    if (st) {
        batch_free(b);
        return st;
    }
    *out = b;
    return RT_OK;
}

extern "C" rt_status rt_batch_run(rt_batch* b, int32_t use_graph, void* stream) {
    if (!b) return fail(RT_ERR_ARG, "rt_batch_run: NULL batch");
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) {
        RT_HIP(batch_enqueue(b, s));
        return RT_OK;
    }
    if (b->captured != plan_version(b->plan)) {  // the plan was re-tuned: capture the step again
        RT_HIP(hipStreamSynchronize(s));
        rt_status st = batch_capture(b);
        if (st) return st;
    }
    RT_HIP(hipGraphLaunch(b->exec, s));
    return RT_OK;
}

extern "C" rt_status rt_batch_plan(rt_batch* b, rt_plan** plan) {
    if (!b || !plan) return fail(RT_ERR_ARG, "rt_batch_plan: NULL argument");
    *plan = b->plan;
    return RT_OK;
}

extern "C" rt_status rt_batch_union(const rt_batch* b, int64_t* points, int64_t* entries) {
    if (!b) return fail(RT_ERR_ARG, "rt_batch_union: NULL batch");
    if (points) *points = b->P_tot;
    if (entries) *entries = b->E_tot;
    return RT_OK;
}

extern "C" rt_status rt_batch_union_index(const rt_batch* b, int32_t* index, void* stream) {
    if (!b || !index) return fail(RT_ERR_ARG, "rt_batch_union_index: NULL argument");
    RT_HIP(hipMemcpyAsync(index, b->uid, sizeof(int32_t) * (size_t)b->P_tot, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
    return RT_OK;
}

extern "C" rt_status rt_batch_destroy(rt_batch* b) {
    if (b) batch_free(b);
    return RT_OK;
}

extern "C" rt_status rt_compute_J_batched(int32_t n_models, const rt_model* const* models, const rt_dirset* set,
                                          const void* const* chi, const void* const* eta, int32_t dtype,
                                          const int64_t* ld, const rt_freq_grid* grid, const double* I_bc,
                                          void* const* J, const rt_solve_opts* opts, void* stream) {
    rt_batch* b = nullptr;
    rt_status st = rt_batch_create(n_models, models, set, chi, eta, dtype, ld, grid, I_bc, J, opts, stream, &b);
    if (st) return st;
    st = rt_batch_run(b, 1, stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    rt_batch_destroy(b);
    if (st) return st;
    if (e != hipSuccess) return hip_fail(e, "rt_compute_J_batched");
    return RT_OK;
}
