// C ABI of the library (declared in include/rt.h): handles, validation,
// workspace planning, launches and HIP-graph plans.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "rt_internal.h"

namespace rt {

namespace {
thread_local std::string g_last_error;

__device__ int32_t g_err_word;

constexpr int MAX_DEVICES = 64;
int32_t* g_err_ptr[MAX_DEVICES] = {nullptr};
int g_cus[MAX_DEVICES] = {0};
int g_xcds[MAX_DEVICES] = {0};
std::mutex g_mu;

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Cache of large device buffers freed by plans (lists, u), per device, so that
// building plan after plan over origin chunks does not map and unmap tens of
// GB each time.  A request takes the smallest cached block of its device that
// is at least as large and at most twice as large (plus 64 MiB); without a fit
// the smaller blocks of its device are freed; blocks beyond POOL_MAX_BYTES held
// in total are freed instead of cached.
struct PoolBlock {
    void* p;
    size_t bytes;
    int dev;
};
std::mutex g_pool_mu;
std::vector<PoolBlock> g_pool;
size_t g_pool_bytes = 0;
std::atomic<int64_t> g_plan_bytes{0};  // bytes of pool_alloc buffers currently owned by plans
constexpr size_t POOL_MIN_BYTES = (size_t)64 << 20;   // smaller buffers go straight to hipMalloc
constexpr size_t POOL_MAX_BYTES = (size_t)32 << 30;

void pool_release_device(int dev) {  // with g_pool_mu held
    for (size_t i = 0; i < g_pool.size();) {
        if (g_pool[i].dev == dev) {
            (void)hipFree(g_pool[i].p);
            g_pool_bytes -= g_pool[i].bytes;
            g_pool[i] = g_pool.back();
            g_pool.pop_back();
        } else {
            ++i;
        }
    }
}
}  // namespace

static hipError_t pool_alloc_(void** ptr, size_t bytes);

// Buffer of at least `bytes` (exactly the requested size is what the caller may use).
hipError_t pool_alloc(void** ptr, size_t bytes) {
    const hipError_t e = pool_alloc_(ptr, bytes);
    if (e == hipSuccess) g_plan_bytes += (int64_t)bytes;
    return e;
}

static hipError_t pool_alloc_(void** ptr, size_t bytes) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (bytes >= POOL_MIN_BYTES) {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        size_t best = g_pool.size();
        for (size_t i = 0; i < g_pool.size(); ++i) {
            const PoolBlock& b = g_pool[i];
            if (b.dev == dev && b.bytes >= bytes && b.bytes <= 2 * bytes + POOL_MIN_BYTES &&
                (best == g_pool.size() || b.bytes < g_pool[best].bytes))
                best = i;
        }
        if (best < g_pool.size()) {
            *ptr = g_pool[best].p;
            g_pool_bytes -= g_pool[best].bytes;
            g_pool[best] = g_pool.back();
            g_pool.pop_back();
            return hipSuccess;
        }
        // no fit: the blocks too small for this request go back to the device
        for (size_t i = 0; i < g_pool.size();) {
            if (g_pool[i].dev == dev && g_pool[i].bytes < bytes) {
                (void)hipFree(g_pool[i].p);
                g_pool_bytes -= g_pool[i].bytes;
                g_pool[i] = g_pool.back();
                g_pool.pop_back();
            } else {
                ++i;
            }
        }
    }
    e = hipMalloc(ptr, bytes);
    if (e == hipErrorOutOfMemory) {  // give the cached blocks back and try once more
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            pool_release_device(dev);
        }
        e = hipMalloc(ptr, bytes);
    }
    return e;
}

// Return a buffer from pool_alloc on device `dev`.  The caller guarantees no work still uses it.
void pool_free(void* ptr, size_t bytes, int dev) {
    if (!ptr) return;
    g_plan_bytes -= (int64_t)bytes;
    if (bytes < POOL_MIN_BYTES) {
        (void)hipFree(ptr);
        return;
    }
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (g_pool_bytes + bytes > POOL_MAX_BYTES) {
        (void)hipFree(ptr);
        return;
    }
    g_pool.push_back(PoolBlock{ptr, bytes, dev});
    g_pool_bytes += bytes;
}

void set_error(const std::string& msg) { g_last_error = msg; }

rt_status fail(rt_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

rt_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return RT_ERR_HIP;
}

int32_t* error_word() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_err_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_err_word)) != hipSuccess) return nullptr;
        if (hipMemset(p, 0, sizeof(int32_t)) != hipSuccess) return nullptr;
        g_err_ptr[dev] = (int32_t*)p;
    }
    return g_err_ptr[dev];
}

int num_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return 256;
    if (!g_cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        g_cus[dev] = v;
    }
    return g_cus[dev];
}

int num_xcds() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return 1;
    if (!g_xcds[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || v <= 0) v = 1;
        g_xcds[dev] = v;
    }
    return g_xcds[dev];
}

}  // namespace rt

using namespace rt;

// ------------------------------------------------------------------ basics

extern "C" const char* rt_last_error(void) { return g_last_error.c_str(); }

extern "C" rt_status rt_version(int32_t* major, int32_t* minor) {
    if (!major || !minor) return fail(RT_ERR_ARG, "rt_version: NULL output");
    *major = 0;
    *minor = 2;
    return RT_OK;
}

extern "C" rt_status rt_struct_sizes(size_t* solve_opts, size_t* freq_grid) {
    if (!solve_opts || !freq_grid) return fail(RT_ERR_ARG, "rt_struct_sizes: NULL output");
    *solve_opts = sizeof(rt_solve_opts);
    *freq_grid = sizeof(rt_freq_grid);
    return RT_OK;
}

// ------------------------------------------------------------------ direction sets

rt_status rt_dirset::ensure_device() {
    int d = 0;
    RT_HIP(hipGetDevice(&d));
    if (dev.dirs && dev.device == d) return RT_OK;
    if (n_origins > 0) return fail(RT_ERR_STATE, "adaptive direction set used on another device");
    if (dev.dirs) {
        (void)hipFree(dev.dirs);
        (void)hipFree(dev.w2);
        dev.dirs = dev.w2 = nullptr;
    }
    RT_HIP(hipMalloc((void**)&dev.dirs, sizeof(double) * dirs.size()));
    RT_HIP(hipMalloc((void**)&dev.w2, sizeof(double) * w2.size()));
    RT_HIP(hipMemcpy(dev.dirs, dirs.data(), sizeof(double) * dirs.size(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(dev.w2, w2.data(), sizeof(double) * w2.size(), hipMemcpyHostToDevice));
    dev.device = d;
    return RT_OK;
}

static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
static int32_t log2i(int64_t v) {
    int32_t l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

extern "C" rt_status rt_dirset_uniform(int32_t nside, rt_dirset** out) {
    if (!out) return fail(RT_ERR_ARG, "rt_dirset_uniform: NULL output");
    *out = nullptr;
    if (!is_pow2(nside) || log2i(nside) > RT_MAX_LEVEL)
        return fail(RT_ERR_UNSUPPORTED, "rt_dirset_uniform: nside must be a power of two <= 2^13");
    auto* s = new rt_dirset();
    s->lmin = s->lmax = log2i(nside);
    const int64_t npix = 12 * (int64_t)nside * nside;
    s->R = 6 * (int64_t)nside * nside;
    s->pix.reserve(s->R);
    for (int64_t p = 0; p < npix; ++p) {
        if (hp_antipode(nside, p) <= p) continue;
        double v[3];
        hp_centre(nside, p, v, nullptr);
        s->pix.push_back(p);
        s->level.push_back(s->lmax);
        s->dirs.insert(s->dirs.end(), v, v + 3);
        s->w2.push_back(2.0 / (double)npix);
    }
    if ((int64_t)s->pix.size() != s->R) {
        delete s;
        return fail(RT_ERR_STATE, "rt_dirset_uniform: internal pair count mismatch");
    }
    *out = s;
    return RT_OK;
}

extern "C" rt_status rt_dirset_info(const rt_dirset* set, int64_t* pairs, int64_t* n_origins, int32_t* lmin,
                                    int32_t* lmax) {
    if (!set) return fail(RT_ERR_ARG, "rt_dirset_info: NULL set");
    if (pairs) *pairs = set->R;
    if (n_origins) *n_origins = set->n_origins;
    if (lmin) *lmin = set->lmin;
    if (lmax) *lmax = set->lmax;
    return RT_OK;
}

extern "C" rt_status rt_dirset_export(const rt_dirset* set, int64_t* pix, int32_t* level, double* dirs, double* w2,
                                      void* stream) {
    if (!set) return fail(RT_ERR_ARG, "rt_dirset_export: NULL set");
    if (set->n_origins == 0) {
        if (pix) std::memcpy(pix, set->pix.data(), sizeof(int64_t) * set->R);
        if (level) std::memcpy(level, set->level.data(), sizeof(int32_t) * set->R);
        if (dirs) std::memcpy(dirs, set->dirs.data(), sizeof(double) * 3 * set->R);
        if (w2) std::memcpy(w2, set->w2.data(), sizeof(double) * set->R);
        return RT_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)set->n_origins * set->R;
    RT_HIP(hipStreamSynchronize(s));
    if (pix) RT_HIP(hipMemcpy(pix, set->dev_pix, sizeof(int64_t) * n, hipMemcpyDeviceToHost));
    if (level) RT_HIP(hipMemcpy(level, set->dev_level, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    if (dirs) RT_HIP(hipMemcpy(dirs, set->dev.dirs, sizeof(double) * 3 * n, hipMemcpyDeviceToHost));
    if (w2) RT_HIP(hipMemcpy(w2, set->dev.w2, sizeof(double) * n, hipMemcpyDeviceToHost));
    return RT_OK;
}

extern "C" rt_status rt_dirset_destroy(rt_dirset* set) {
    if (!set) return RT_OK;
    if (set->dev.dirs) (void)hipFree(set->dev.dirs);
    if (set->dev.w2) (void)hipFree(set->dev.w2);
    if (set->dev_pix) (void)hipFree(set->dev_pix);
    if (set->dev_level) (void)hipFree(set->dev_level);
    delete set;
    return RT_OK;
}

// ------------------------------------------------------------------ model

extern "C" rt_status rt_model_create(const double* pos, int64_t P, const int64_t* nbr_off, const int32_t* nbr_idx,
                                     int64_t E, const float* vel, void* stream, rt_model** out) {
    return model_create(pos, P, nbr_off, nbr_idx, E, vel, nullptr, true, (hipStream_t)stream, out);
}

rt_status rt::model_create(const double* pos, int64_t P, const int64_t* nbr_off, const int32_t* nbr_idx, int64_t E,
                           const float* vel, const int32_t* key, bool morton_rows, hipStream_t s, rt_model** out) {
    if (!out) return fail(RT_ERR_ARG, "rt_model_create: NULL output");
    *out = nullptr;
    if (!pos || !nbr_off || (E > 0 && !nbr_idx) || P <= 0 || E < 0)
        return fail(RT_ERR_ARG, "rt_model_create: NULL array or non-positive size");
    if (P > INT32_MAX || E > INT32_MAX)
        return fail(RT_ERR_UNSUPPORTED, "rt_model_create: more than 2^31-1 points or neighbour entries");
    auto* m = new rt_model();
    m->pos = pos;
    m->P = P;
    m->off = nbr_off;
    m->idx = nbr_idx;
    m->E = E;
    m->vel = vel;
    RT_HIP(hipGetDevice(&m->device));
    int32_t* bad = nullptr;
    hipError_t e = hipMalloc((void**)&m->nbr, sizeof(NbrRec) * (size_t)std::max<int64_t>(E, 1));
    if (e == hipSuccess) e = hipMalloc((void**)&m->nid, sizeof(int32_t) * (size_t)std::max<int64_t>(E, 1));
    if (e == hipSuccess) e = hipMalloc((void**)&m->rows, sizeof(int2) * (size_t)P);
    if (e == hipSuccess) e = hipMalloc((void**)&bad, sizeof(int32_t));
    if (e == hipSuccess) e = launch_fill_i32(bad, 1, 0, s);
    if (e == hipSuccess) e = launch_check_model(m, bad, s);
    int32_t hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (bad) (void)hipFree(bad);
    if (e == hipSuccess && !hbad) {  // a valid CSR: build the records
        // rows in the Morton order of the points, so that the rows a walk reads next are near
        // in memory (the positions' host copy is kept for the plans' origin orders)
        std::vector<int32_t> lay;
        int32_t* lay_d = nullptr;
        void* ws = nullptr;
        if (morton_rows) {
            std::lock_guard<std::mutex> lk(m->host_mu);
            m->host_pos.resize((size_t)P * 3);
            e = hipMemcpyAsync(m->host_pos.data(), pos, sizeof(double) * m->host_pos.size(), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) morton_order_host(m->host_pos.data(), P, nullptr, P, lay, nullptr, 0);
            else m->host_pos.clear();
            if (e == hipSuccess) e = hipMalloc((void**)&lay_d, sizeof(int32_t) * (size_t)P);
            if (e == hipSuccess)
                e = hipMemcpyAsync(lay_d, lay.data(), sizeof(int32_t) * (size_t)P, hipMemcpyHostToDevice, s);
        }
        if (e == hipSuccess) e = hipMalloc(&ws, build_nbr_workspace(P));
        if (e == hipSuccess) e = launch_build_nbr(m, key, lay_d, ws, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (lay_d) (void)hipFree(lay_d);
        if (ws) (void)hipFree(ws);
    }
    if (e != hipSuccess) {
        rt_status st = hip_fail(e, "rt_model_create");
        if (m->nbr) (void)hipFree(m->nbr);
        if (m->nid) (void)hipFree(m->nid);
        if (m->rows) (void)hipFree(m->rows);
        delete m;
        return st;
    }
    if (hbad) {
        if (m->nbr) (void)hipFree(m->nbr);
        if (m->nid) (void)hipFree(m->nid);
        if (m->rows) (void)hipFree(m->rows);
        delete m;
        return fail(hbad == 8 ? RT_ERR_ARG : RT_ERR_MESH, std::string("rt_model_create: invalid model (") +
                                     ((hbad & 1) ? "index out of range " : "") + ((hbad & 2) ? "bad offsets " : "") +
                                     ((hbad & 4) ? "self neighbour " : "") +
                                     ((hbad & 8) ? "position not finite or beyond 1e150" : "") + ")");
    }
    *out = m;
    return RT_OK;
}

extern "C" rt_status rt_model_destroy(rt_model* m) {
    if (!m) return RT_OK;
    if (m->nbr) (void)hipFree(m->nbr);
    if (m->nid) (void)hipFree(m->nid);
    if (m->rows) (void)hipFree(m->rows);
    delete m;
    return RT_OK;
}

extern "C" rt_status rt_validate_host(const double* pos, int64_t P, const int64_t* off, const int32_t* idx, int64_t E,
                                      const void* chi, int32_t dtype, int64_t F, int64_t ld) {
    if (!pos || !off || (E > 0 && !idx) || P <= 0 || E < 0) return fail(RT_ERR_ARG, "rt_validate_host: bad arguments");
    for (int64_t i = 0; i < 3 * P; ++i)
        if (!std::isfinite(pos[i])) return fail(RT_ERR_MESH, "rt_validate_host: non-finite position");
    if (off[0] != 0 || off[P] != E) return fail(RT_ERR_MESH, "rt_validate_host: offsets must run from 0 to E");
    std::vector<std::pair<int32_t, int32_t>> edges;
    edges.reserve((size_t)E);
    for (int64_t p = 0; p < P; ++p) {
        if (off[p + 1] < off[p]) return fail(RT_ERR_MESH, "rt_validate_host: offsets not monotone");
        for (int64_t e = off[p]; e < off[p + 1]; ++e) {
            int32_t k = idx[e];
            if (k < 0 || k >= P) return fail(RT_ERR_MESH, "rt_validate_host: neighbour index out of range");
            if (k == p) return fail(RT_ERR_MESH, "rt_validate_host: self neighbour");
            edges.emplace_back((int32_t)p, k);
        }
    }
    std::sort(edges.begin(), edges.end());
    for (size_t i = 1; i < edges.size(); ++i)
        if (edges[i] == edges[i - 1]) return fail(RT_ERR_MESH, "rt_validate_host: duplicate neighbour");
    for (auto& pr : edges)
        if (!std::binary_search(edges.begin(), edges.end(), std::make_pair(pr.second, pr.first)))
            return fail(RT_ERR_MESH, "rt_validate_host: neighbour lists are not symmetric");
    if (chi) {
        if (F <= 0 || ld < F) return fail(RT_ERR_ARG, "rt_validate_host: need 0 < F <= ld");
        if (F > 4096) return fail(RT_ERR_UNSUPPORTED, "rt_validate_host: more than 4096 frequencies");
        for (int64_t p = 0; p < P; ++p)
            for (int64_t f = 0; f < F; ++f) {
                double c = dtype == RT_F32 ? (double)((const float*)chi)[p * ld + f] : ((const double*)chi)[p * ld + f];
                if (!(c > 0.0) || !std::isfinite(c)) return fail(RT_ERR_OPACITY, "rt_validate_host: chi must be finite and > 0");
            }
    }
    return RT_OK;
}

// ------------------------------------------------------------------ tracing

static rt_status check_trace_args(const rt_model* m, rt_dirset* set, int64_t n_origins, const char* who) {
    if (!m || !set) return fail(RT_ERR_ARG, std::string(who) + ": NULL model or set");
    if (n_origins < 0) return fail(RT_ERR_ARG, std::string(who) + ": negative origin count");
    if (set->n_origins > 0 && set->n_origins != n_origins)
        return fail(RT_ERR_ARG, std::string(who) + ": adaptive set built for a different number of origins");
    return set->ensure_device();
}

extern "C" rt_status rt_trace_count_workspace(const rt_dirset* set, int64_t n_origins, size_t* bytes) {
    if (!set || !bytes || n_origins < 0) return fail(RT_ERR_ARG, "rt_trace_count_workspace: bad arguments");
    const int64_t n = n_origins * 2 * set->R;
    *bytes = align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1)) + align_up(scan_workspace(n));
    return RT_OK;
}

extern "C" rt_status rt_trace_count(const rt_model* m, const rt_dirset* set_, const int32_t* origins, int64_t n_origins,
                                    int64_t* ray_off, void* ws, size_t ws_bytes, void* stream) {
    rt_dirset* set = const_cast<rt_dirset*>(set_);
    rt_status st = check_trace_args(m, set, n_origins, "rt_trace_count");
    if (st) return st;
    if (!ray_off) return fail(RT_ERR_ARG, "rt_trace_count: NULL ray_off");
    size_t need = 0;
    rt_trace_count_workspace(set, n_origins, &need);
    if (!ws || ws_bytes < need) return fail(RT_ERR_CAPACITY, "rt_trace_count: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = n_origins * 2 * set->R;
    int32_t* lens = (int32_t*)ws;
    void* scan_ws = (char*)ws + align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
    RT_HIP(launch_trace_count(m, origins, n_origins, set->R, set->d_dirs(), set->n_origins > 0, lens, s));
    RT_HIP(launch_scan(lens, n, ray_off, scan_ws, s));
    return RT_OK;
}

extern "C" rt_status rt_trace_write(const rt_model* m, const rt_dirset* set_, const int32_t* origins, int64_t n_origins,
                                    const int64_t* ray_off, int32_t* ray_ids, double* ray_Z, int64_t capacity,
                                    void* stream) {
    rt_dirset* set = const_cast<rt_dirset*>(set_);
    rt_status st = check_trace_args(m, set, n_origins, "rt_trace_write");
    if (st) return st;
    if (!ray_off || (capacity > 0 && (!ray_ids || !ray_Z)) || capacity < 0)
        return fail(RT_ERR_ARG, "rt_trace_write: NULL list or negative capacity");
    if (!error_word()) return fail(RT_ERR_HIP, "rt_trace_write: no device error word");
    RT_HIP(launch_trace_write(m, origins, n_origins, set->R, set->d_dirs(), set->n_origins > 0, ray_off, ray_ids,
                              ray_Z, capacity, (hipStream_t)stream));
    return RT_OK;
}

extern "C" rt_status rt_trace(const rt_model* m, const rt_dirset* set_, const int32_t* origins, int64_t n_origins,
                              int64_t* ray_off, int32_t* ray_ids, double* ray_Z, int64_t capacity, int64_t* total_dev,
                              void* ws, size_t ws_bytes, void* stream) {
    rt_dirset* set = const_cast<rt_dirset*>(set_);
    rt_status st = check_trace_args(m, set, n_origins, "rt_trace");
    if (st) return st;
    if (!ray_off || !total_dev || capacity < 0 || (capacity > 0 && (!ray_ids || !ray_Z)))
        return fail(RT_ERR_ARG, "rt_trace: NULL output or negative capacity");
    size_t need = 0;
    rt_trace_count_workspace(set, n_origins, &need);
    if (!ws || ws_bytes < need) return fail(RT_ERR_CAPACITY, "rt_trace: workspace too small");
    if (!error_word()) return fail(RT_ERR_HIP, "rt_trace: no device error word");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = n_origins * 2 * set->R;
    int32_t* lens = (int32_t*)ws;
    void* scan_ws = (char*)ws + align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
    RT_HIP(launch_trace_count(m, origins, n_origins, set->R, set->d_dirs(), set->n_origins > 0, lens, s));
    RT_HIP(launch_scan(lens, n, ray_off, scan_ws, s));
    RT_HIP(hipMemcpyAsync(total_dev, ray_off + n, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    RT_HIP(launch_trace_write(m, origins, n_origins, set->R, set->d_dirs(), set->n_origins > 0, ray_off, ray_ids,
                              ray_Z, capacity, s));
    return RT_OK;
}

// ------------------------------------------------------------------ solve

rt_solve_opts rt::default_solve_opts() {
    rt_solve_opts o;
    std::memset(&o, 0, sizeof(o));
    o.precision = RT_F32;
    o.schedule = RT_SCHED_DIRECT;
    o.waves_per_cu = 0;
    o.n_bins = 0;
    o.bins_per_octave = 0;
    o.group = 0;
    o.trace_lanes = 0;
    o.padded_trace_budget = 0;
    o.walk = RT_WALK_EXACT;
    o.dtau_max = 0.0;
    o.max_substeps = 0;
    o.dv_max = 0.0;
    o.scheme = RT_SCHEME_FEAUTRIER2;
    return o;
}

static rt_solve_opts default_opts() { return default_solve_opts(); }

int32_t rt::opts_bins(const rt_solve_opts& o) { return o.n_bins > 0 ? std::min(o.n_bins, 128) : 64; }
int32_t rt::opts_bins_per_octave(const rt_solve_opts& o) { return o.bins_per_octave > 0 ? o.bins_per_octave : 4; }
static bool valid_bins_per_octave(int32_t v) { return v == 0 || v == 1 || v == 2 || v == 4 || v == 8; }

static size_t solve_ws_bytes(int64_t n_origins, int64_t R, int64_t F, const rt_solve_opts& o, bool need_u) {
    const size_t es = o.precision == RT_F64 ? 8 : 4;
    const int64_t n_items = n_origins * R * ((F + 63) / 64);
    size_t b = 0;
    if (need_u) b += align_up(es * (size_t)std::max<int64_t>(n_origins * R * F, 1));
    if (o.schedule == RT_SCHED_BINNED) b += align_up(bin_workspace(n_items, opts_bins(o))) + 256;
    return b;
}

extern "C" rt_status rt_solve_workspace(const rt_dirset* set, int64_t n_origins, int64_t F, const rt_solve_opts* opts,
                                        size_t* bytes) {
    if (!set || !bytes || n_origins < 0 || F <= 0) return fail(RT_ERR_ARG, "rt_solve_workspace: bad arguments");
    rt_solve_opts o = opts ? *opts : default_opts();
    *bytes = solve_ws_bytes(n_origins, set->R, F, o, true);
    return RT_OK;
}

rt_status rt::fill_solve_launch(const rt_model* m, rt_dirset* set, const int32_t* origins, int64_t n_origins,
                                const int64_t* ray_off, const int32_t* ray_ids, const double* ray_Z, const void* chi,
                                const void* eta, int32_t dtype, int64_t ld, const rt_freq_grid* grid,
                                const double* I_bc, void* J, const rt_solve_opts& o, SolveLaunch& a) {
    if (!m || !set || !chi || !eta || !grid || !I_bc || (!J && n_origins > 0))
        return fail(RT_ERR_ARG, "solve: NULL argument");
    if (o.precision != RT_F32 && o.precision != RT_F64) return fail(RT_ERR_ARG, "solve: precision must be RT_F32 or RT_F64");
    if (dtype != o.precision) return fail(RT_ERR_ARG, "solve: table dtype must match the precision");
    if (grid->n_blocks < 1 || grid->n_blocks > RT_MAX_FREQ_BLOCKS || !grid->len || !grid->dx)
        return fail(RT_ERR_UNSUPPORTED, "solve: 1 .. 8 frequency blocks required");
    std::memset(&a, 0, sizeof(a));
    int64_t F = 0;
    for (int b = 0; b < grid->n_blocks; ++b) {
        if (grid->len[b] <= 0 || !(grid->dx[b] > 0.0)) return fail(RT_ERR_ARG, "solve: block lengths and dx must be > 0");
        a.blk_start[b] = (int32_t)F;
        a.inv_dx[b] = 1.0 / grid->dx[b];
        a.dx[b] = grid->dx[b];
        F += grid->len[b];
    }
    for (int b = grid->n_blocks; b <= RT_MAX_FREQ_BLOCKS; ++b) a.blk_start[b] = (int32_t)F;
    if (F > 4096) return fail(RT_ERR_UNSUPPORTED, "solve: more than 4096 frequencies");
    if (ld < F) return fail(RT_ERR_ARG, "solve: ld < F");
    if (set->n_origins > 0 && set->n_origins != n_origins)
        return fail(RT_ERR_ARG, "solve: adaptive set built for a different number of origins");
    rt_status st = set->ensure_device();
    if (st) return st;
    a.origins = origins;
    a.n_origins = n_origins;
    a.R = set->R;
    a.dirs = set->d_dirs();
    a.w2 = set->d_w2();
    a.per_origin = set->n_origins > 0;
    a.ray_off = ray_off;
    a.ray_ids = ray_ids;
    a.ray_Z = ray_Z;
    a.chi = chi;
    a.eta = eta;
    a.ld = ld;
    a.F = (int32_t)F;
    a.n_blocks = grid->n_blocks;
    a.vel = m->vel;
    a.P = m->P;
    a.I_bc = I_bc;
    a.J = J;
    if (!(o.dtau_max >= 0.0) || !(o.dv_max >= 0.0) || o.max_substeps < 0)
        return fail(RT_ERR_ARG, "solve: dtau_max, dv_max and max_substeps must be >= 0");
    if (!valid_bins_per_octave(o.bins_per_octave))
        return fail(RT_ERR_ARG, "solve: bins_per_octave must be 1, 2, 4 or 8 (0 = 4)");
    a.dtau_max_rcp = o.dtau_max > 0.0 ? 1.0 / o.dtau_max : 0.0;
    a.dv_max_rcp = o.dv_max > 0.0 && m->vel ? 1.0 / o.dv_max : 0.0;
    a.max_sub = o.max_substeps > 0 ? o.max_substeps : 1024;
    a.schedule = o.schedule;
    a.n_bins = opts_bins(o);
    a.bins_per_octave = opts_bins_per_octave(o);
    int wpc = o.waves_per_cu > 0 ? std::min(o.waves_per_cu, MAX_WAVES_PER_CU) : 32;
    a.grid_waves = num_cus() * wpc;
    a.n_xcd = num_xcds();
    if (o.group != 0 && o.group != 4 && o.group != 8) return fail(RT_ERR_ARG, "solve: group must be 4 or 8");
    a.group = o.group ? o.group : 4;
    if (o.scheme != RT_SCHEME_FEAUTRIER2 && o.scheme != RT_SCHEME_HERMITE)
        return fail(RT_ERR_ARG, "solve: scheme must be RT_SCHEME_FEAUTRIER2 or RT_SCHEME_HERMITE");
    a.scheme = o.scheme;
    {  // every byte offset into chi and eta (row * ld + column) fits in 32 bits
        const double tbytes = (double)m->P * (double)ld * (double)(dtype == RT_F64 ? 8 : 4);
        a.small_tables = tbytes < 4294967296.0 ? 1 : 0;
    }
    a.err = error_word();
    if (!a.err) return fail(RT_ERR_HIP, "solve: no device error word");
    return RT_OK;
}

// Carve the solve scratch out of ws: u (unless given), then bins and the queue counter.
static rt_status carve_solve_ws(SolveLaunch& a, const rt_solve_opts& o, void* u_out, void* ws, size_t ws_bytes,
                                void** bin_ws) {
    const bool need_u = u_out == nullptr;
    size_t need = solve_ws_bytes(a.n_origins, a.R, a.F, o, need_u);
    if (need > 0 && (!ws || ws_bytes < need)) return fail(RT_ERR_CAPACITY, "solve: workspace too small");
    char* p = (char*)ws;
    const size_t es = o.precision == RT_F64 ? 8 : 4;
    if (need_u) {
        a.u = p;
        p += align_up(es * (size_t)std::max<int64_t>(a.n_origins * a.R * a.F, 1));
    } else {
        a.u = u_out;
    }
    *bin_ws = nullptr;
    if (o.schedule == RT_SCHED_BINNED) {
        a.queue = (int32_t*)p;
        p += 256;
        *bin_ws = p;
    }
    return RT_OK;
}

static hipError_t enqueue_solve(SolveLaunch& a, int precision, void* bin_ws, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (a.schedule == RT_SCHED_BINNED) {
        int32_t* items = nullptr;
        e = launch_bin(a, bin_ws, &items, s);
        if (e != hipSuccess) return e;
        a.items = items;
        e = launch_fill_i32(a.queue, 1, 0, s);
        if (e != hipSuccess) return e;
    }
    e = launch_solve(a, precision, s);
    if (e != hipSuccess) return e;
    return launch_reduce(a, precision, s);
}

extern "C" rt_status rt_solve(const rt_model* m, const rt_dirset* set_, const int32_t* origins, int64_t n_origins,
                              const int64_t* ray_off, const int32_t* ray_ids, const double* ray_Z, const void* chi,
                              const void* eta, int32_t dtype, int64_t ld, const rt_freq_grid* grid, const double* I_bc,
                              void* J, void* u_out, const rt_solve_opts* opts, void* ws, size_t ws_bytes,
                              void* stream) {
    rt_dirset* set = const_cast<rt_dirset*>(set_);
    rt_solve_opts o = opts ? *opts : default_opts();
    if (o.schedule != RT_SCHED_DIRECT && o.schedule != RT_SCHED_BINNED)
        return fail(RT_ERR_ARG, "rt_solve: schedule must be RT_SCHED_DIRECT or RT_SCHED_BINNED (spatial: plans only)");
    if (!ray_off) return fail(RT_ERR_ARG, "rt_solve: NULL ray_off");
    SolveLaunch a;
    rt_status st = fill_solve_launch(m, set, origins, n_origins, ray_off, ray_ids, ray_Z, chi, eta, dtype, ld, grid,
                                     I_bc, J, o, a);
    if (st) return st;
    if (n_origins * a.R * ((a.F + 63) / 64) > MAX_SOLVE_ITEMS)
        return fail(RT_ERR_UNSUPPORTED, "rt_solve: too many work items");
    void* bin_ws = nullptr;
    st = carve_solve_ws(a, o, u_out, ws, ws_bytes, &bin_ws);
    if (st) return st;
    RT_HIP(enqueue_solve(a, o.precision, bin_ws, (hipStream_t)stream));
    return RT_OK;
}

// ------------------------------------------------------------------ solve without allocation

namespace {
// Scratch of rt_solve_noalloc: the per-pair u and the length bins.  Each device
// holds its own copy from the time the library's code is loaded on it until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
void* g_scratch_ptr[MAX_DEVICES] = {nullptr};
}  // namespace

// Device address of the current device's scratch, looked up once per device.
static rt_status noalloc_scratch(void** out) {
    int dev = 0;
    RT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(RT_ERR_UNSUPPORTED, "rt_solve_noalloc: device index too large");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        RT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(RT_ERR_HIP, "rt_solve_noalloc: no address for the static scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RT_OK;
}

extern "C" rt_status rt_solve_noalloc(const rt_model* m, const rt_dirset* set_, const int32_t* origins,
                                      int64_t n_origins, const int64_t* ray_off, const int32_t* ray_ids,
                                      const double* ray_Z, const void* chi, const void* eta, int32_t dtype, int64_t ld,
                                      const rt_freq_grid* grid, const double* I_bc, void* J, void* u_out,
                                      const rt_solve_opts* opts, void* stream) {
    rt_dirset* set = const_cast<rt_dirset*>(set_);
    rt_solve_opts o = opts ? *opts : default_opts();
    if (o.schedule != RT_SCHED_DIRECT && o.schedule != RT_SCHED_BINNED)
        return fail(RT_ERR_ARG, "rt_solve_noalloc: schedule must be RT_SCHED_DIRECT or RT_SCHED_BINNED");
    if (!ray_off) return fail(RT_ERR_ARG, "rt_solve_noalloc: NULL ray_off");
    if (set) {  // a shared set uploads its tables on first use on a device: that must have happened already
        int dev = -1;
        RT_HIP(hipGetDevice(&dev));
        if (!set->dev.dirs || set->dev.device != dev)
            return fail(RT_ERR_STATE, "rt_solve_noalloc: the direction set's tables are not on this device yet "
                                      "(use the set once with an allocating call, e.g. rt_trace_count)");
    }
    SolveLaunch a;
    rt_status st = fill_solve_launch(m, set, origins, n_origins, ray_off, ray_ids, ray_Z, chi, eta, dtype, ld, grid,
                                     I_bc, J, o, a);
    if (st) return st;
    if (n_origins * a.R * ((a.F + 63) / 64) > MAX_SOLVE_ITEMS)
        return fail(RT_ERR_UNSUPPORTED, "rt_solve_noalloc: too many work items");
    const size_t need = solve_ws_bytes(n_origins, a.R, a.F, o, u_out == nullptr);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(RT_ERR_CAPACITY, "rt_solve_noalloc: " + std::to_string(need) +
                                         " bytes of scratch needed, above the static 64 MiB; pass u_out or "
                                         "solve fewer origins per call");
    void* ws = nullptr;
    st = noalloc_scratch(&ws);
    if (st) return st;
    void* bin_ws = nullptr;
    st = carve_solve_ws(a, o, u_out, ws, NOALLOC_SCRATCH_BYTES, &bin_ws);
    if (st) return st;
    RT_HIP(enqueue_solve(a, o.precision, bin_ws, (hipStream_t)stream));
    return RT_OK;
}

extern "C" rt_status rt_sync_status(void* stream) {
    RT_HIP(hipStreamSynchronize((hipStream_t)stream));
    int32_t* w = error_word();
    if (!w) return fail(RT_ERR_HIP, "rt_sync_status: no device error word");
    int32_t h = 0;
    RT_HIP(hipMemcpy(&h, w, sizeof(int32_t), hipMemcpyDeviceToHost));
    RT_HIP(hipMemset(w, 0, sizeof(int32_t)));
    // the first error in this order is returned; the message lists every latched one
    std::string all;
    if (h & ERRBIT_CAPACITY) all += " [ray list capacity]";
    if (h & ERRBIT_STEP) all += " [fourth-order step limit]";
    if (h & ERRBIT_NONFINITE) all += " [non-finite u]";
    if (h & ERRBIT_ORIGIN) all += " [origin id out of range]";
    if (h & ERRBIT_CAPACITY) return fail(RT_ERR_CAPACITY, "a ray list exceeded its capacity; latched:" + all);
    if (h & ERRBIT_STEP)
        return fail(RT_ERR_STEP,
                    "a fourth-order row met an optical-depth step beyond its limit (about 3.46); latched:" + all);
    if (h & ERRBIT_NONFINITE) return fail(RT_ERR_NONFINITE, "the solve produced a non-finite u; latched:" + all);
    if (h & ERRBIT_ORIGIN) return fail(RT_ERR_ARG, "an origin id was outside 0 .. P-1; latched:" + all);
    return RT_OK;
}

// ------------------------------------------------------------------ plans

struct rt_plan {
    const rt_model* m = nullptr;
    rt_dirset* set = nullptr;
    const int32_t* origins = nullptr;
    int64_t n_origins = 0;
    int64_t n_rays = 0;
    int64_t total = 0;
    rt_solve_opts o;
    SolveLaunch a;
    int32_t* lens = nullptr;
    int64_t* ray_off = nullptr;
    int32_t* ids = nullptr;
    double* Z = nullptr;
    void* scan_ws = nullptr;
    void* solve_ws = nullptr;
    void* bin_ws = nullptr;
    int32_t* bin_items = nullptr;  // the length-binned item order (inside bin_buf), built by plan_configure
    // single-pass tracing into padded slots (cap per ray), then compaction
    int64_t cap = 0;
    int32_t* pids = nullptr;
    double* pZ = nullptr;
    // spatial schedule: origin order (Morton), built on first use
    int32_t* order = nullptr;
    // exact-slot walks: per direction, windows of that order sorted by ray length (from the
    // creation-time count pass); null when it could not be allocated
    int32_t* walk_order = nullptr;
    // the sweep's per-pair orders ([R][n_origins]; uniform sets), built on first use of the spatial
    // schedule over the segments below (one by default: the model's bounding sphere)
    int32_t* pair_order = nullptr;
    std::vector<OrderSeg> segs;
    // the solve launch as filled from the caller's arguments, before any schedule is applied
    SolveLaunch base;
    void* u_buf = nullptr;
    void* bin_buf = nullptr;   // binned schedule: queue counter + bins, allocated on first use
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool exact = false;  // RT_WALK_EXACT: walk straight into the creation-time slots
    int64_t version = 0; // incremented whenever the graph is re-captured
    // bytes of the cached large buffers (ids, Z, padded slots, u)
    size_t ids_bytes = 0, Z_bytes = 0, pids_bytes = 0, pZ_bytes = 0, u_bytes = 0;
};

// Stages: 0 count, 1 scan, 2 write, 3 bin (+ queue reset), 4 sweep, 5 reduce.
// With `ev` (7 events) each stage is bracketed by event records.
static hipError_t plan_enqueue(rt_plan* p, hipStream_t s, hipEvent_t* ev = nullptr) {
    hipError_t e = hipSuccess;
    auto mark = [&](int i) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[i], s);
    };
    const int per = p->set->n_origins > 0;
    mark(0);
    if (p->exact) {  // one walk straight into the creation-time slots
        if (e == hipSuccess)
            e = launch_trace_write(p->m, p->origins, p->n_origins, p->set->R, p->set->d_dirs(), per, p->ray_off,
                                   p->ids, p->Z, p->total, s, p->order, p->o.trace_lanes, p->walk_order);
        mark(1);
        mark(2);
    } else {
    if (e == hipSuccess) {
        if (p->pids)
            e = launch_trace_padded(p->m, p->origins, p->n_origins, p->set->R, p->set->d_dirs(), per, p->lens, p->pids,
                                    p->pZ, p->cap, s, p->order, p->o.trace_lanes);
        else
            e = launch_trace_count(p->m, p->origins, p->n_origins, p->set->R, p->set->d_dirs(), per, p->lens, s,
                                   p->order, p->o.trace_lanes);
    }
    mark(1);
    if (e == hipSuccess) e = launch_scan(p->lens, p->n_rays, p->ray_off, p->scan_ws, s);
    mark(2);
    if (e == hipSuccess) {
        if (p->pids)
            e = launch_compact(p->pids, p->pZ, p->cap, p->ray_off, p->n_rays, p->ids, p->Z, s);
        else
            e = launch_trace_write(p->m, p->origins, p->n_origins, p->set->R, p->set->d_dirs(), per, p->ray_off,
                                   p->ids, p->Z, p->total, s, p->order, p->o.trace_lanes);
    }
    }
    mark(3);
    SolveLaunch a = p->a;
    if (e == hipSuccess && a.schedule == RT_SCHED_BINNED) {  // the binned order was built when configured
        a.items = p->bin_items;
        e = launch_fill_i32(a.queue, 1, 0, s);
    }
    mark(4);
    if (e == hipSuccess) e = launch_solve(a, p->o.precision, s);
    mark(5);
    if (e == hipSuccess) e = launch_reduce(a, p->o.precision, s);
    mark(6);
    return e;
}

static void plan_free(rt_plan* p) {
    // the cached buffers may be handed to the next plan at once: no work of this one may still run
    // (hipFree, which the small buffers go through, waits for the device the same way)
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (void* q : {(void*)p->lens, (void*)p->ray_off, p->scan_ws, p->solve_ws, (void*)p->order, p->bin_buf,
                    (void*)p->pair_order, (void*)p->walk_order})
        if (q) (void)hipFree(q);
    const int dev = p->m->device;
    pool_free(p->ids, p->ids_bytes, dev);
    pool_free(p->Z, p->Z_bytes, dev);
    pool_free(p->pids, p->pids_bytes, dev);
    pool_free(p->pZ, p->pZ_bytes, dev);
    pool_free(p->u_buf, p->u_bytes, dev);
    delete p;
}

// Origin positions in the order of the Morton (Z-order) code of their points:
// 21 bits per axis over the bounding box of the origins (of each segment's
// origins, when segments are given; segments keep their order).
hipError_t rt::morton_order(const rt_model* m, const int32_t* origins, int64_t n_o, hipStream_t s,
                            std::vector<int32_t>& order, const int64_t* seg, int n_seg) {
    std::lock_guard<std::mutex> lk(m->host_mu);
    std::vector<double>& pos = m->host_pos;
    std::vector<int32_t> org;
    hipError_t e = hipSuccess;
    if (pos.empty()) {
        pos.resize((size_t)m->P * 3);
        e = hipMemcpyAsync(pos.data(), m->pos, sizeof(double) * pos.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            pos.clear();
            return e;
        }
    }
    if (e == hipSuccess && origins) {
        org.resize((size_t)n_o);
        e = hipMemcpyAsync(org.data(), origins, sizeof(int32_t) * org.size(), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    morton_order_host(pos.data(), m->P, origins ? org.data() : nullptr, n_o, order, seg, n_seg);
    return hipSuccess;
}

void rt::morton_order_host(const double* pos, int64_t P, const int32_t* org, int64_t n_o, std::vector<int32_t>& order,
                           const int64_t* seg, int n_seg) {
    auto pt = [&](int64_t k) -> int64_t {
        int64_t o = org ? (int64_t)org[(size_t)k] : k;
        return (o < 0 || o >= P) ? 0 : o;
    };
    auto spread = [](uint64_t v) {  // 21 bits -> every third bit
        v &= 0x1fffff;
        v = (v | v << 32) & 0x1f00000000ffffULL;
        v = (v | v << 16) & 0x1f0000ff0000ffULL;
        v = (v | v << 8) & 0x100f00f00f00f00fULL;
        v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
        v = (v | v << 2) & 0x1249249249249249ULL;
        return v;
    };
    order.resize((size_t)n_o);
    for (int64_t k = 0; k < n_o; ++k) order[(size_t)k] = (int32_t)k;
    const int64_t whole[2] = {0, n_o};
    if (n_seg <= 0 || !seg) {
        seg = whole;
        n_seg = 1;
    }
    std::vector<std::pair<uint64_t, int32_t>> key;
    for (int g = 0; g < n_seg; ++g) {
        const int64_t k0 = std::max<int64_t>(0, seg[g]), k1 = std::min<int64_t>(n_o, seg[g + 1]);
        if (k1 <= k0) continue;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t k = k0; k < k1; ++k)
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::min(lo[c], pos[(size_t)(3 * pt(k) + c)]);
                hi[c] = std::max(hi[c], pos[(size_t)(3 * pt(k) + c)]);
            }
        key.resize((size_t)(k1 - k0));
        for (int64_t k = k0; k < k1; ++k) {
            uint64_t code = 0;
            for (int c = 0; c < 3; ++c) {
                double w = hi[c] > lo[c] ? (pos[(size_t)(3 * pt(k) + c)] - lo[c]) / (hi[c] - lo[c]) : 0.0;
                uint64_t qv = (uint64_t)std::min(std::max(w * 2097151.0, 0.0), 2097151.0);
                code |= spread(qv) << c;
            }
            key[(size_t)(k - k0)] = {code, (int32_t)k};
        }
        std::sort(key.begin(), key.end());
        for (int64_t k = k0; k < k1; ++k) order[(size_t)k] = key[(size_t)(k - k0)].second;
    }
}

extern "C" rt_status rt_spatial_order(const rt_model* m, const int32_t* origins, int64_t n_origins, int32_t* order,
                                      void* stream) {
    if (!m || n_origins < 0 || (n_origins > 0 && !order)) return fail(RT_ERR_ARG, "rt_spatial_order: bad arguments");
    if (n_origins == 0) return RT_OK;
    std::vector<int32_t> ord;
    RT_HIP(morton_order(m, origins, n_origins, (hipStream_t)stream, ord));
    std::memcpy(order, ord.data(), sizeof(int32_t) * ord.size());
    return RT_OK;
}

// Apply scheduling options to a plan whose lists and u buffer exist: build what
// the schedule needs on first use (spatial origin order, bin workspace) and
// re-capture the whole step as one graph on a private stream (the caller's
// stream may be the legacy default stream, which cannot be captured).

// The sweep's per-pair orders of a plan over a uniform set (order.hip), built once; skipped
// (Morton order for every pair) for per-origin sets, when they would take more than 2 GiB,
// for more than 65 535 segments, and when the device memory for them is not there.
// Without given segments the model's points' bounding sphere is the one segment.
static hipError_t plan_pair_orders(rt_plan* p) {
    if (p->pair_order || p->n_origins <= 0 || p->set->n_origins > 0) return hipSuccess;
    const int64_t R = p->set->R, n = p->n_origins;
    if ((double)R * (double)n * 4.0 > 2147483648.0 || p->segs.size() > 65535) return hipSuccess;
    std::vector<OrderSeg> segs = p->segs;
    if (segs.empty()) {
        std::lock_guard<std::mutex> lk(p->m->host_mu);
        std::vector<double>& hp = p->m->host_pos;
        if (hp.empty()) {
            hp.resize((size_t)p->m->P * 3);
            hipError_t e = hipMemcpy(hp.data(), p->m->pos, sizeof(double) * hp.size(), hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                hp.clear();
                return e;
            }
        }
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t q = 0; q < p->m->P; ++q)
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::min(lo[c], hp[(size_t)(3 * q + c)]);
                hi[c] = std::max(hi[c], hp[(size_t)(3 * q + c)]);
            }
        OrderSeg g;
        g.end = n;
        double r2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            g.c[c] = 0.5 * (lo[c] + hi[c]);
            r2 += 0.25 * (hi[c] - lo[c]) * (hi[c] - lo[c]);
        }
        g.rho = std::sqrt(r2);
        segs.push_back(g);
    }
    std::vector<double> dirs((size_t)(3 * R));
    hipError_t e = hipMemcpy(dirs.data(), p->set->d_dirs(), sizeof(double) * dirs.size(), hipMemcpyDeviceToHost);
    OrderSeg* dsegs = nullptr;
    void* ws = nullptr;
    int32_t* out = nullptr;
    if (e == hipSuccess) e = hipMalloc((void**)&dsegs, sizeof(OrderSeg) * segs.size());
    if (e == hipSuccess)
        e = hipMemcpy(dsegs, segs.data(), sizeof(OrderSeg) * segs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&ws, pair_order_workspace(n));
    if (e == hipSuccess) e = hipMalloc((void**)&out, sizeof(int32_t) * (size_t)(R * n));
    if (e == hipSuccess)
        e = build_pair_orders(p->m->pos, p->m->P, p->origins, n, dirs.data(), R, dsegs, (int)segs.size(), out, ws,
                              p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (dsegs) (void)hipFree(dsegs);
    if (ws) (void)hipFree(ws);
    if (e != hipSuccess) {
        if (out) (void)hipFree(out);
        if (e == hipErrorOutOfMemory) {  // an optimisation only: the sweep keeps the Morton order
            (void)hipGetLastError();
            return hipSuccess;
        }
        return e;
    }
    p->pair_order = out;
    return hipSuccess;
}

static rt_status plan_configure(rt_plan* p, const rt_solve_opts& o) {
    if (o.schedule < RT_SCHED_DIRECT || o.schedule > RT_SCHED_SPATIAL) return fail(RT_ERR_ARG, "plan: bad schedule");
    if (o.group != 0 && o.group != 4 && o.group != 8) return fail(RT_ERR_ARG, "plan: group must be 4 or 8");
    if (o.trace_lanes != 0 && o.trace_lanes != 4 && o.trace_lanes != 8 && o.trace_lanes != 16)
        return fail(RT_ERR_ARG, "plan: trace_lanes must be 4, 8 or 16");
    if (!valid_bins_per_octave(o.bins_per_octave)) return fail(RT_ERR_ARG, "plan: bins_per_octave must be 1, 2, 4 or 8");
    hipError_t e = hipSuccess;
    const rt_solve_opts prev = p->o;
    p->o.schedule = o.schedule;
    p->o.group = o.group;
    p->o.trace_lanes = o.trace_lanes;
    p->o.waves_per_cu = o.waves_per_cu;
    p->o.n_bins = o.n_bins;
    p->o.bins_per_octave = o.bins_per_octave;
    SolveLaunch a = p->base;
    a.u = p->u_buf;
    a.schedule = o.schedule == RT_SCHED_BINNED ? RT_SCHED_BINNED : RT_SCHED_DIRECT;
    a.group = o.group ? o.group : 4;
    a.n_bins = opts_bins(o);
    a.bins_per_octave = opts_bins_per_octave(o);
    a.grid_waves = num_cus() * (o.waves_per_cu > 0 ? std::min(o.waves_per_cu, MAX_WAVES_PER_CU) : 32);
    a.items = nullptr;
    a.order = nullptr;
    a.queue = nullptr;
    p->bin_ws = nullptr;
    p->bin_items = nullptr;
    // The walk always runs direction-major over Morton-ordered origins (best L2
    // reuse whatever the sweep's schedule); the spatial schedule applies the same
    // order to the sweep's items.
    if (p->n_origins > 0 && !p->order) {
        std::vector<int32_t> ord;
        e = morton_order(p->m, p->origins, p->n_origins, p->stream, ord);
        if (e == hipSuccess) e = hipMalloc((void**)&p->order, sizeof(int32_t) * ord.size());
        if (e == hipSuccess) e = hipMemcpy(p->order, ord.data(), sizeof(int32_t) * ord.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            p->o = prev;
            return hip_fail(e, "plan: spatial order");
        }
    }
    // the spatial schedule walks the sweep's items direction by direction, each pair's
    // items in that pair's line order (Morton order of the origins when there is none);
    // the binned schedule uses the Morton order inside each length bin
    if (o.schedule == RT_SCHED_SPATIAL || o.schedule == RT_SCHED_BINNED) a.order = p->order;
    if (o.schedule == RT_SCHED_SPATIAL) {
        e = plan_pair_orders(p);
        if (e != hipSuccess) {
            p->o = prev;
            return hip_fail(e, "plan: pair orders");
        }
        a.pair_order = p->pair_order;
    }
    if (o.schedule == RT_SCHED_BINNED) {
        const size_t need = align_up(bin_workspace(solve_items(a), 128)) + 256;
        if (!p->bin_buf) {
            e = hipMalloc(&p->bin_buf, need);
            if (e != hipSuccess) {
                p->o = prev;
                return hip_fail(e, "plan: bin workspace");
            }
        }
        a.queue = (int32_t*)p->bin_buf;
        p->bin_ws = (char*)p->bin_buf + 256;
        // Ray lengths are fixed for the plan's life (the count pass at creation gave ray_off, and every walk
        // of the plan reproduces them), so the length-binned item order is built once here, not per replay.
        e = launch_bin(a, p->bin_ws, &p->bin_items, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) {
            p->o = prev;
            return hip_fail(e, "plan: binned order");
        }
    }
    p->a = a;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = plan_enqueue(p, cap);
        e = hipStreamEndCapture(cap, &p->graph);
        if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return hip_fail(e, "plan: graph capture");
    ++p->version;
    return RT_OK;
}

hipError_t rt::plan_enqueue_step(rt_plan* p, hipStream_t s) { return plan_enqueue(p, s); }
int64_t rt::plan_version(const rt_plan* p) { return p->version; }

extern "C" rt_status rt_plan_retune(rt_plan* p, const rt_solve_opts* opts, void* stream) {
    if (!p || !opts) return fail(RT_ERR_ARG, "rt_plan_retune: NULL argument");
    RT_HIP(hipStreamSynchronize((hipStream_t)stream));
    p->stream = (hipStream_t)stream;
    return plan_configure(p, *opts);
}

extern "C" rt_status rt_plan_create(const rt_model* m, const rt_dirset* set_, const int32_t* origins, int64_t n_origins,
                                    const void* chi, const void* eta, int32_t dtype, int64_t ld,
                                    const rt_freq_grid* grid, const double* I_bc, void* J, const rt_solve_opts* opts,
                                    void* stream, rt_plan** out) {
    return plan_create_ordered(m, const_cast<rt_dirset*>(set_), origins, n_origins, chi, eta, dtype, ld, grid, I_bc, J,
                               opts, (hipStream_t)stream, nullptr, out);
}

rt_status rt::plan_create_ordered(const rt_model* m, rt_dirset* set, const int32_t* origins, int64_t n_origins,
                                  const void* chi, const void* eta, int32_t dtype, int64_t ld, const rt_freq_grid* grid,
                                  const double* I_bc, void* J, const rt_solve_opts* opts, hipStream_t stream,
                                  const std::vector<int32_t>* given_order, rt_plan** out,
                                  const std::vector<OrderSeg>* segs) {
    if (!out) return fail(RT_ERR_ARG, "rt_plan_create: NULL output");
    *out = nullptr;
    rt_status st = check_trace_args(m, set, n_origins, "rt_plan_create");
    if (st) return st;
    if (opts && (opts->schedule < RT_SCHED_DIRECT || opts->schedule > RT_SCHED_SPATIAL))
        return fail(RT_ERR_ARG, "rt_plan_create: bad schedule");
    if (opts && (opts->walk < RT_WALK_EXACT || opts->walk > RT_WALK_TWO_PASS))
        return fail(RT_ERR_ARG, "rt_plan_create: bad walk mode");
    hipStream_t s = (hipStream_t)stream;
    auto* p = new rt_plan();
    p->m = m;
    p->set = set;
    p->origins = origins;
    p->n_origins = n_origins;
    p->n_rays = n_origins * 2 * set->R;
    p->o = opts ? *opts : default_opts();
    if (segs) p->segs = *segs;
    hipError_t e = hipMalloc((void**)&p->lens, sizeof(int32_t) * (size_t)std::max<int64_t>(p->n_rays, 1));
    if (e == hipSuccess) e = hipMalloc((void**)&p->ray_off, sizeof(int64_t) * (size_t)(p->n_rays + 1));
    if (e == hipSuccess) e = hipMalloc(&p->scan_ws, scan_workspace(p->n_rays));
    // the walk's origin order (Morton), used by the count pass here and by every walk of the plan
    if (e == hipSuccess && n_origins > 0) {
        std::vector<int32_t> ord;
        if (given_order && (int64_t)given_order->size() == n_origins)
            ord = *given_order;
        else
            e = morton_order(m, origins, n_origins, s, ord);
        if (e == hipSuccess) e = hipMalloc((void**)&p->order, sizeof(int32_t) * ord.size());
        if (e == hipSuccess) e = hipMemcpy(p->order, ord.data(), sizeof(int32_t) * ord.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
        e = launch_trace_count(m, origins, n_origins, set->R, set->d_dirs(), set->n_origins > 0, p->lens, s, p->order,
                               p->o.trace_lanes);
    if (e == hipSuccess) e = launch_scan(p->lens, p->n_rays, p->ray_off, p->scan_ws, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&p->total, p->ray_off + p->n_rays, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    p->ids_bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(p->total, 1);
    p->Z_bytes = sizeof(double) * (size_t)std::max<int64_t>(p->total, 1);
    if (e == hipSuccess) e = pool_alloc((void**)&p->ids, p->ids_bytes);
    if (e == hipSuccess) e = pool_alloc((void**)&p->Z, p->Z_bytes);
    p->exact = p->o.walk == RT_WALK_EXACT;
    // the exact walk's ray order: each direction's windows of the origin order sorted by ray length
    // (a schedule only: without it the walk takes the origin order itself)
    if (e == hipSuccess && p->exact && p->order && p->n_rays > 0) {
        if (hipMalloc((void**)&p->walk_order, sizeof(int32_t) * (size_t)p->n_rays) == hipSuccess) {
            e = launch_length_order(p->lens, p->order, n_origins, set->R, p->walk_order, s);
        } else {
            (void)hipGetLastError();
            p->walk_order = nullptr;
        }
    }
    // Longest ray: the padded single-pass walk is used when its slots fit the budget.
    int32_t longest = 0;
    if (e == hipSuccess && p->n_rays > 0 && p->o.walk == RT_WALK_PADDED) {
        std::vector<int32_t> hl((size_t)p->n_rays);
        e = hipMemcpyAsync(hl.data(), p->lens, sizeof(int32_t) * hl.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        for (int32_t v : hl) longest = std::max(longest, v);
    }
    const size_t pad_bytes = (size_t)p->n_rays * (size_t)std::max(longest, 1) * 12;
    const size_t budget = opts && opts->padded_trace_budget > 0 ? (size_t)opts->padded_trace_budget
                                                               : (size_t)32 << 30;
    if (e == hipSuccess && p->n_rays > 0 && p->o.walk == RT_WALK_PADDED && !(opts && opts->padded_trace_budget < 0) &&
        pad_bytes <= budget) {
        p->cap = std::max(longest, 1);
        p->pids_bytes = sizeof(int32_t) * (size_t)p->n_rays * p->cap;
        p->pZ_bytes = sizeof(double) * (size_t)p->n_rays * p->cap;
        e = pool_alloc((void**)&p->pids, p->pids_bytes);
        if (e == hipSuccess) e = pool_alloc((void**)&p->pZ, p->pZ_bytes);
    }
    if (e != hipSuccess) {
        st = hip_fail(e, "rt_plan_create");
        plan_free(p);
        return st;
    }
    st = fill_solve_launch(m, set, origins, n_origins, p->ray_off, p->ids, p->Z, chi, eta, dtype, ld, grid, I_bc, J, p->o,
                     p->a);
    if (!st && solve_items(p->a) > MAX_SOLVE_ITEMS) st = fail(RT_ERR_UNSUPPORTED, "rt_plan_create: too many work items");
    if (st) {
        plan_free(p);
        return st;
    }
    p->base = p->a;
    const size_t es = p->o.precision == RT_F64 ? 8 : 4;
    p->u_bytes = es * (size_t)std::max<int64_t>(n_origins * set->R * p->a.F, 1);
    e = pool_alloc(&p->u_buf, p->u_bytes);
    if (e != hipSuccess) {
        st = hip_fail(e, "rt_plan_create: u buffer");
        plan_free(p);
        return st;
    }
    p->stream = s;
    st = plan_configure(p, p->o);
    if (st) {
        plan_free(p);
        return st;
    }
    *out = p;
    return RT_OK;
}

extern "C" rt_status rt_plan_run(rt_plan* p, int32_t use_graph, void* stream) {
    if (!p) return fail(RT_ERR_ARG, "rt_plan_run: NULL plan");
    hipStream_t s = (hipStream_t)stream;
    if (use_graph) {
        RT_HIP(hipGraphLaunch(p->exec, s));
    } else {
        RT_HIP(plan_enqueue(p, s));
    }
    return RT_OK;
}

extern "C" rt_status rt_plan_profile(rt_plan* p, int32_t n_runs, double* stage_ms, void* stream) {
    if (!p || !stage_ms || n_runs <= 0) return fail(RT_ERR_ARG, "rt_plan_profile: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[7] = {};
    for (auto& x : ev) RT_HIP(hipEventCreate(&x));
    double acc[6] = {0, 0, 0, 0, 0, 0};
    hipError_t e = hipSuccess;
    for (int r = 0; r < n_runs && e == hipSuccess; ++r) {
        e = plan_enqueue(p, s, ev);
        if (e == hipSuccess) e = hipEventSynchronize(ev[6]);
        for (int i = 0; i < 6 && e == hipSuccess; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            acc[i] += ms;
        }
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(e, "rt_plan_profile");
    for (int i = 0; i < 6; ++i) stage_ms[i] = acc[i] / n_runs;
    return RT_OK;
}

extern "C" rt_status rt_plan_info(const rt_plan* p, int64_t* total, const int64_t** ray_off, const int32_t** ray_ids,
                                  const double** ray_Z) {
    if (!p) return fail(RT_ERR_ARG, "rt_plan_info: NULL plan");
    if (total) *total = p->total;
    if (ray_off) *ray_off = p->ray_off;
    if (ray_ids) *ray_ids = p->ids;
    if (ray_Z) *ray_Z = p->Z;
    return RT_OK;
}

extern "C" rt_status rt_plan_copy_rays(const rt_plan* p, int64_t* ray_off, int32_t* ray_ids, double* ray_Z,
                                       void* stream) {
    if (!p || !ray_off || (p->total > 0 && (!ray_ids || !ray_Z))) return fail(RT_ERR_ARG, "rt_plan_copy_rays: NULL");
    hipStream_t s = (hipStream_t)stream;
    RT_HIP(hipMemcpyAsync(ray_off, p->ray_off, sizeof(int64_t) * (size_t)(p->n_rays + 1), hipMemcpyDeviceToDevice, s));
    if (p->total > 0) {
        RT_HIP(hipMemcpyAsync(ray_ids, p->ids, sizeof(int32_t) * (size_t)p->total, hipMemcpyDeviceToDevice, s));
        RT_HIP(hipMemcpyAsync(ray_Z, p->Z, sizeof(double) * (size_t)p->total, hipMemcpyDeviceToDevice, s));
    }
    return RT_OK;
}

extern "C" rt_status rt_plan_copy_u(const rt_plan* p, void* u, void* stream) {
    if (!p || (!u && p->n_origins > 0)) return fail(RT_ERR_ARG, "rt_plan_copy_u: NULL");
    const size_t es = p->o.precision == RT_F64 ? 8 : 4;
    const size_t n = (size_t)p->n_origins * (size_t)p->set->R * (size_t)p->a.F;
    if (n > 0) RT_HIP(hipMemcpyAsync(u, p->u_buf, es * n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return RT_OK;
}

extern "C" rt_status rt_plan_destroy(rt_plan* p) {
    if (p) plan_free(p);
    return RT_OK;
}

extern "C" rt_status rt_release_cached_memory(void) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (const PoolBlock& b : g_pool) (void)hipFree(b.p);
    g_pool.clear();
    g_pool_bytes = 0;
    return RT_OK;
}

extern "C" rt_status rt_plan_memory(size_t* bytes) {
    if (!bytes) return fail(RT_ERR_ARG, "rt_plan_memory: NULL output");
    const int64_t v = g_plan_bytes.load();
    *bytes = v > 0 ? (size_t)v : 0;
    return RT_OK;
}

extern "C" rt_status rt_cached_memory(size_t* bytes) {
    if (!bytes) return fail(RT_ERR_ARG, "rt_cached_memory: NULL output");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    *bytes = g_pool_bytes;
    return RT_OK;
}

// ------------------------------------------------------------------ autotuner

static std::string tune_signature(const rt_model* m, const rt_dirset* set, int64_t n_origins, int64_t F,
                                  const rt_solve_opts& o) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char& c : arch)
        if (c == ' ' || c == ':') c = '_';
    char buf[256];
    // the sweep's kernel variant: rows of the scheme, refined lines (optical depth, velocity)
    const int refine = (o.dtau_max > 0.0 ? 1 : 0) | (o.dv_max > 0.0 && m->vel ? 2 : 0);
    std::snprintf(buf, sizeof(buf), "%s_P%lld_E%lld_R%lld_n%lld_F%lld_p%d_v%d_a%d_s%d_r%d", arch.c_str(),
                  (long long)m->P, (long long)m->E, (long long)set->R, (long long)n_origins, (long long)F,
                  (int)o.precision, m->vel ? 1 : 0, set->n_origins > 0 ? 1 : 0, (int)o.scheme, refine);
    return buf;
}

// The candidate search on a configured plan: each candidate run varies the
// walk's lanes per ray and the sweep's schedule parameters (they act on
// different stages, and the HIP-event stage times credit them separately).
// Leaves the plan re-captured with the chosen options.
static rt_status tune_plan(rt_plan* p, int32_t n_runs, int32_t verbose, hipStream_t stream, rt_solve_opts* best,
                           double* best_ms) {
    if (n_runs <= 0) n_runs = 2;
    const int lanes[3] = {4, 8, 16};
    struct SweepCand { int sc, gr, wpc, bins, bpo; };
    const SweepCand sw[9] = {{RT_SCHED_SPATIAL, 4, 0, 0, 0},  {RT_SCHED_SPATIAL, 8, 0, 0, 0},
                             {RT_SCHED_BINNED, 8, 32, 64, 4}, {RT_SCHED_BINNED, 8, 32, 32, 2},
                             {RT_SCHED_BINNED, 4, 16, 128, 4}, {RT_SCHED_DIRECT, 4, 0, 0, 0},
                             {RT_SCHED_BINNED, 8, 32, 128, 8}, {RT_SCHED_BINNED, 8, 64, 64, 4},
                             {RT_SCHED_DIRECT, 8, 0, 0, 0}};
    const rt_solve_opts b0 = p->o;
    rt_solve_opts o = b0;
    rt_status st = RT_OK;
    double walk_best = 1e300, sweep_best = 1e300, other = 0.0, walk_default = 0.0, sweep_default = 0.0;
    int lane_best = 4;
    SweepCand sw_best = sw[0];
    for (int i = 0; i < 9 && !st; ++i) {
        o.schedule = sw[i].sc;
        o.group = sw[i].gr;
        o.waves_per_cu = sw[i].wpc;
        o.n_bins = sw[i].bins;
        o.bins_per_octave = sw[i].bpo;
        o.trace_lanes = lanes[i % 3];
        st = plan_configure(p, o);
        if (st) break;
        double ms[6];
        st = rt_plan_profile(p, 1, ms, stream);  // warm-up
        if (!st) st = rt_plan_profile(p, n_runs, ms, stream);
        if (st) break;
        const double walk = ms[0] + ms[2], sweep = ms[3] + ms[4];
        if (i == 0) {  // the library defaults: spatial schedule, group 4, 4 lanes
            walk_default = walk;
            sweep_default = sweep;
        }
        if (i < 3 && walk < walk_best) {
            walk_best = walk;
            lane_best = lanes[i];
        }
        if (sweep < sweep_best) {
            sweep_best = sweep;
            sw_best = sw[i];
        }
        other = ms[1] + ms[5];
        if (verbose)
            std::fprintf(stderr,
                         "autotune: lanes %d schedule %d group %d waves/CU %d bins %d per octave %d -> walk %.3f ms, "
                         "sweep %.3f ms\n",
                         o.trace_lanes, o.schedule, o.group, o.waves_per_cu, o.n_bins, opts_bins_per_octave(o), walk,
                         sweep);
    }
    if (st) return st;
    // keep a default unless a candidate beats it by 5%: choices closer than that swap from box to box
    if (!(walk_best < 0.95 * walk_default)) {
        lane_best = 4;
        walk_best = walk_default;
    }
    if (!(sweep_best < 0.95 * sweep_default)) {
        sw_best = sw[0];
        sweep_best = sweep_default;
    }
    *best = b0;
    best->schedule = sw_best.sc;
    best->group = sw_best.gr;
    best->waves_per_cu = sw_best.wpc;
    best->n_bins = sw_best.bins;
    best->bins_per_octave = sw_best.bpo;
    best->trace_lanes = lane_best;
    if (best_ms) *best_ms = walk_best + sweep_best + other;
    return plan_configure(p, *best);
}

extern "C" rt_status rt_autotune_plan(rt_plan* p, int32_t n_runs, int32_t verbose, void* stream, rt_solve_opts* best,
                                      double* best_ms) {
    if (!p || !best) return fail(RT_ERR_ARG, "rt_autotune_plan: NULL argument");
    RT_HIP(hipStreamSynchronize((hipStream_t)stream));
    p->stream = (hipStream_t)stream;
    return tune_plan(p, n_runs, verbose, (hipStream_t)stream, best, best_ms);
}

extern "C" rt_status rt_autotune(const rt_model* m, const rt_dirset* set, const int32_t* origins, int64_t n_origins,
                                 const void* chi, const void* eta, int32_t dtype, int64_t ld,
                                 const rt_freq_grid* grid, const double* I_bc, void* J, const rt_solve_opts* base,
                                 int32_t n_runs, const char* cache_path, int32_t verbose, void* stream,
                                 rt_solve_opts* best, double* best_ms) {
    if (!m || !set || !grid || !best) return fail(RT_ERR_ARG, "rt_autotune: NULL argument");
    rt_solve_opts b0 = base ? *base : default_opts();
    int64_t F = 0;
    for (int i = 0; i < grid->n_blocks && grid->len; ++i) F += grid->len[i];
    const std::string sig = tune_signature(m, set, n_origins, F, b0);
    if (cache_path && *cache_path) {
        FILE* f = std::fopen(cache_path, "r");
        if (f) {
            char key[256];
            int sc, gr, la, wpc, nb, bpo;
            double ms;
            while (std::fscanf(f, "%255s %d %d %d %d %d %d %lf", key, &sc, &gr, &la, &wpc, &nb, &bpo, &ms) == 8) {
                if (sig == key) {
                    *best = b0;
                    best->schedule = sc;
                    best->group = gr;
                    best->trace_lanes = la;
                    best->waves_per_cu = wpc;
                    best->n_bins = nb;
                    best->bins_per_octave = bpo;
                    if (best_ms) *best_ms = ms;
                    std::fclose(f);
                    return RT_OK;
                }
            }
            std::fclose(f);
        }
    }
    rt_plan* p = nullptr;
    rt_solve_opts o = b0;
    o.schedule = RT_SCHED_SPATIAL;
    o.group = 4;
    o.trace_lanes = 4;
    rt_status st = rt_plan_create(m, set, origins, n_origins, chi, eta, dtype, ld, grid, I_bc, J, &o, stream, &p);
    if (st) return st;
    double bms = 0.0;
    st = tune_plan(p, n_runs, verbose, (hipStream_t)stream, best, &bms);
    rt_plan_destroy(p);
    if (st) return st;
    if (best_ms) *best_ms = bms;
    if (cache_path && *cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f, "%s %d %d %d %d %d %d %.6f\n", sig.c_str(), best->schedule, best->group, best->trace_lanes,
                         best->waves_per_cu, best->n_bins, best->bins_per_octave, bms);
            std::fclose(f);
        }
    }
    return RT_OK;
}

// ------------------------------------------------------------------ adaptive sets (see dirset.hip)
