// Adaptive HEALPix direction sets (Section 2.1.3, Fig. 1).
//
// Per origin, the directions to a sample of points are histogrammed at level
// lmax, the histogram is downgraded through the nested hierarchy (a coarse
// pixel is the union of its four children), the count of an antipodal pair is
// the sum over both pixels, and starting from every pair at lmin the top half
// of the active pairs of each level (count descending, ties to the smaller
// canonical ring index) is refined into the pairs of their children; the rest,
// and every pair reaching lmax, are leaves.  Every origin gets the same number
// of pairs, 6*4^lmin*((2^K - 1)/2 + 2^K), K = lmax - lmin.
//
// One workgroup per origin.  The level histograms, the active pairs and the
// leaves live in LDS (lmax <= 4 keeps it under 64 KB).  Pixel lookup of a
// direction uses a square root and arctangent built from IEEE +, -, *, / in a
// fixed order (file contract off), so boundary directions are classified
// exactly as any other evaluation of the same steps; direction vectors and
// weights of the leaves come from host-built tables (the same values as the
// uniform sets).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rt_internal.h"

#pragma clang fp contract(off)

namespace rt {

namespace {

constexpr int DS_MAX_LEVELS = 5;  // lmin .. lmax with lmax <= 4
constexpr int DS_BLOCK = 256;

__host__ __device__ inline double fx_sqrt(double x) {
    if (!(x > 0.0)) return 0.0;
    uint64_t u = __builtin_bit_cast(uint64_t, x);
    u = (u >> 1) + 0x1FF8000000000000ULL;  // halve the exponent: a seed within ~6%
    double y = __builtin_bit_cast(double, u);
    for (int i = 0; i < 6; ++i) y = 0.5 * (y + x / y);
    return y;
}

__host__ __device__ inline double fx_atan2(double y, double x) {
    const double ax = fabs(x), ay = fabs(y);
    if (ax == 0.0 && ay == 0.0) return 0.0;
    const bool swap = ay > ax;
    const double mx = swap ? ay : ax, mn = swap ? ax : ay;
    double t = mn / mx, base = 0.0;
    if (t > 0.41421356237309503) {  // beyond tan(pi/8): atan(t) = pi/4 + atan((t-1)/(t+1))
        t = (t - 1.0) / (t + 1.0);
        base = 0.78539816339744831;
    }
    const double t2 = t * t;
    double p = 0.0;
    for (int k = 21; k >= 0; --k) {  // Taylor series of atan to t^43, Horner in t^2
        const double c = ((k & 1) ? -1.0 : 1.0) / (double)(2 * k + 1);
        p = p * t2 + c;
    }
    double r = base + t * p;
    if (swap) r = 1.5707963267948966 - r;
    if (x < 0.0) r = 3.1415926535897931 - r;
    if (y < 0.0) r = -r;
    return r;
}

// Ring-scheme pixel of the direction of (vx, vy, vz) at resolution nside.
__host__ __device__ inline int64_t fx_vec2pix(int64_t nside, double vx, double vy, double vz) {
    const int64_t npix = 12 * nside * nside;
    const int64_t ncap = 2 * nside * (nside - 1);
    const double r = fx_sqrt((vx * vx + vy * vy) + vz * vz);
    const double z = vz / r;
    double phi = fx_atan2(vy, vx);
    if (phi < 0.0) phi = phi + 6.2831853071795862;
    const double za = fabs(z);
    double tt = phi / 1.5707963267948966;
    if (tt >= 4.0) tt = 0.0;
    if (za <= 2.0 / 3.0) {
        const double t1 = (double)nside * (0.5 + tt);
        const double t2 = (double)nside * z * 0.75;
        const int64_t jp = (int64_t)floor(t1 - t2);
        const int64_t jm = (int64_t)floor(t1 + t2);
        const int64_t ir = nside + 1 + jp - jm;
        const int64_t kshift = 1 - (ir & 1);
        int64_t ip = (jp + jm - nside + kshift + 1) / 2;
        ip = ((ip % (4 * nside)) + 4 * nside) % (4 * nside);
        return ncap + (ir - 1) * 4 * nside + ip;
    }
    const double tp = tt - floor(tt);
    const double tmp = (double)nside * fx_sqrt(3.0 * (1.0 - za));
    const int64_t jp = (int64_t)floor(tp * tmp);
    const int64_t jm = (int64_t)floor((1.0 - tp) * tmp);
    const int64_t ir = jp + jm + 1;
    int64_t ip = (int64_t)floor(tt * (double)ir);
    ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
    if (z > 0.0) return 2 * ir * (ir - 1) + ip;
    return npix - 2 * ir * (ir + 1) + ip;
}

struct DsTables {
    int L;      // levels lmin .. lmax
    int lmin;
    int64_t R;  // pairs per origin
    int npix[DS_MAX_LEVELS];
    int hoff[DS_MAX_LEVELS];       // offset of each level's histogram in LDS
    int act_max;                   // largest active set
    const int32_t* anti[DS_MAX_LEVELS];
    const int32_t* child[DS_MAX_LEVELS];  // [npix][4], levels 0 .. L-2
    const double* cen[DS_MAX_LEVELS];     // [npix][3]
};

__global__ __launch_bounds__(DS_BLOCK) void k_dirset(const double* __restrict__ pos, int64_t P,
                                                      const int32_t* __restrict__ origins,
                                                      const int32_t* __restrict__ sample, int64_t n_sample,
                                                      const DsTables t, int64_t* __restrict__ out_pix,
                                                      int32_t* __restrict__ out_level, double* __restrict__ out_dirs,
                                                      double* __restrict__ out_w2, int32_t* __restrict__ err) {
    extern __shared__ int32_t sm[];
    int32_t* hist = sm;                                     // all levels
    int32_t* a_pix = sm + t.hoff[t.L - 1] + t.npix[t.L - 1];  // active pairs (pixel, count, rank)
    int32_t* a_cnt = a_pix + t.act_max;
    int32_t* a_rank = a_cnt + t.act_max;
    int32_t* n_pix = a_rank + t.act_max;                    // next level's active pairs
    int32_t* lv_pix = n_pix + t.act_max;                    // leaves
    int32_t* lv_lev = lv_pix + t.R;
    const int tid = threadIdx.x;
    const int64_t oi = blockIdx.x;
    const int64_t o = origins ? (int64_t)origins[oi] : oi;
    const int total = t.hoff[t.L - 1] + t.npix[t.L - 1];
    for (int i = tid; i < total; i += DS_BLOCK) hist[i] = 0;
    __syncthreads();
    if (o < 0 || o >= P) {
        if (tid == 0) atomicOr(err, ERRBIT_ORIGIN);
        return;
    }
    const double ox = pos[3 * o], oy = pos[3 * o + 1], oz = pos[3 * o + 2];
    const int64_t nsm = (int64_t)1 << (t.lmin + t.L - 1);
    int32_t* hmax = hist + t.hoff[t.L - 1];
    for (int64_t j = tid; j < n_sample; j += DS_BLOCK) {
        const int64_t s = sample[j];
        if (s == o) continue;
        if (s < 0 || s >= P) {
            atomicOr(err, ERRBIT_ORIGIN);
            continue;
        }
        const double vx = pos[3 * s] - ox, vy = pos[3 * s + 1] - oy, vz = pos[3 * s + 2] - oz;
        if (vx == 0.0 && vy == 0.0 && vz == 0.0) continue;
        atomicAdd(&hmax[fx_vec2pix(nsm, vx, vy, vz)], 1);
    }
    __syncthreads();
    // downgrade: a coarse pixel's count is the sum over its four children
    for (int k = t.L - 2; k >= 0; --k) {
        for (int p = tid; p < t.npix[k]; p += DS_BLOCK) {
            const int32_t* c = t.child[k] + 4 * p;
            const int32_t* hf = hist + t.hoff[k + 1];
            hist[t.hoff[k] + p] = hf[c[0]] + hf[c[1]] + hf[c[2]] + hf[c[3]];
        }
        __syncthreads();
    }
    // level lmin: every canonical pixel (the smaller index of each antipodal pair)
    __shared__ int n_act_s, n_leaf_s;
    if (tid == 0) {
        int n = 0;
        for (int p = 0; p < t.npix[0]; ++p)
            if (t.anti[0][p] > p) a_pix[n++] = p;
        n_act_s = n;
        n_leaf_s = 0;
    }
    __syncthreads();
    for (int k = 0; k < t.L; ++k) {
        const int n_act = n_act_s;
        const int32_t* hk = hist + t.hoff[k];
        for (int i = tid; i < n_act; i += DS_BLOCK) a_cnt[i] = hk[a_pix[i]] + hk[t.anti[k][a_pix[i]]];
        __syncthreads();
        if (k == t.L - 1) {
            for (int i = tid; i < n_act; i += DS_BLOCK) {
                lv_pix[n_leaf_s + i] = a_pix[i];
                lv_lev[n_leaf_s + i] = t.lmin + k;
            }
            __syncthreads();
            break;
        }
        // rank: pairs with a larger count, or an equal count and a smaller index, come first
        for (int i = tid; i < n_act; i += DS_BLOCK) {
            const int ci = a_cnt[i], pi = a_pix[i];
            int r = 0;
            for (int j = 0; j < n_act; ++j) r += (a_cnt[j] > ci) || (a_cnt[j] == ci && a_pix[j] < pi);
            a_rank[i] = r;
        }
        __syncthreads();
        const int half = n_act / 2;
        const int32_t* ak1 = t.anti[k + 1];
        for (int i = tid; i < n_act; i += DS_BLOCK) {
            const int r = a_rank[i];
            if (r < half) {
                const int32_t* c = t.child[k] + 4 * a_pix[i];
#pragma unroll
                for (int q = 0; q < 4; ++q) n_pix[4 * r + q] = c[q] < ak1[c[q]] ? c[q] : ak1[c[q]];
            } else {
                lv_pix[n_leaf_s + (r - half)] = a_pix[i];
                lv_lev[n_leaf_s + (r - half)] = t.lmin + k;
            }
        }
        __syncthreads();
        for (int i = tid; i < 4 * half; i += DS_BLOCK) a_pix[i] = n_pix[i];
        if (tid == 0) {
            n_leaf_s += n_act - half;
            n_act_s = 4 * half;
        }
        __syncthreads();
    }
    // leaves ordered by (level, canonical index)
    const int R = (int)t.R;
    for (int i = tid; i < R; i += DS_BLOCK) {
        const int li = lv_lev[i], pi = lv_pix[i];
        int r = 0;
        for (int j = 0; j < R; ++j) r += (lv_lev[j] < li) || (lv_lev[j] == li && lv_pix[j] < pi);
        const int64_t q = oi * t.R + r;
        const int k = li - t.lmin;
        out_pix[q] = pi;
        out_level[q] = li;
        out_dirs[3 * q] = t.cen[k][3 * pi];
        out_dirs[3 * q + 1] = t.cen[k][3 * pi + 1];
        out_dirs[3 * q + 2] = t.cen[k][3 * pi + 2];
        const double ns = (double)((int64_t)1 << li);
        out_w2[q] = 2.0 / (12.0 * ns * ns);
    }
}

}  // namespace

}  // namespace rt

using namespace rt;

extern "C" rt_status rt_dirset_adaptive(const rt_model* model, int32_t lmin, int32_t lmax,
                                        const int32_t* sample_ids_dev, int64_t n_sample,
                                        const int32_t* origins_dev, int64_t n_origins, void* stream,
                                        rt_dirset** out) {
    if (!out) return fail(RT_ERR_ARG, "rt_dirset_adaptive: NULL output");
    *out = nullptr;
    if (!model || n_origins < 0 || n_sample < 0 || (n_sample > 0 && !sample_ids_dev))
        return fail(RT_ERR_ARG, "rt_dirset_adaptive: bad arguments");
    if (lmin < 0 || lmax < lmin || lmax > 4)
        return fail(RT_ERR_UNSUPPORTED, "rt_dirset_adaptive: need 0 <= lmin <= lmax <= 4");
    hipStream_t s = (hipStream_t)stream;
    const int L = lmax - lmin + 1;
    int64_t R = 0, act = (int64_t)6 << (2 * lmin), act_max = act;
    for (int l = lmin; l < lmax; ++l) {
        R += act / 2;
        act = 4 * (act / 2);
        act_max = std::max(act_max, act);
    }
    R += act;
    // host tables per level: antipodes, children (by the lookup of each fine centre), centres
    DsTables t;
    std::memset(&t, 0, sizeof(t));
    t.L = L;
    t.lmin = lmin;
    t.R = R;
    t.act_max = (int)act_max;
    std::vector<int32_t> ibuf;
    std::vector<double> dbuf;
    std::vector<size_t> anti_off(L), child_off(L), cen_off(L);
    int hoff = 0;
    for (int k = 0; k < L; ++k) {
        const int64_t ns = (int64_t)1 << (lmin + k);
        const int npix = (int)(12 * ns * ns);
        t.npix[k] = npix;
        t.hoff[k] = hoff;
        hoff += npix;
        anti_off[k] = ibuf.size();
        for (int p = 0; p < npix; ++p) ibuf.push_back((int32_t)hp_antipode(ns, p));
        cen_off[k] = dbuf.size();
        for (int p = 0; p < npix; ++p) {
            double v[3];
            hp_centre(ns, p, v, nullptr);
            dbuf.insert(dbuf.end(), v, v + 3);
        }
    }
    for (int k = 0; k + 1 < L; ++k) {
        const int64_t ns = (int64_t)1 << (lmin + k);
        std::vector<int32_t> ch((size_t)t.npix[k] * 4, -1);
        std::vector<int> fill((size_t)t.npix[k], 0);
        for (int c = 0; c < t.npix[k + 1]; ++c) {
            const double* v = &dbuf[cen_off[k + 1] + 3 * (size_t)c];
            const int64_t p = fx_vec2pix(ns, v[0], v[1], v[2]);
            if (fill[(size_t)p] >= 4) return fail(RT_ERR_STATE, "rt_dirset_adaptive: hierarchy is not 4-to-1");
            ch[4 * (size_t)p + fill[(size_t)p]++] = c;
        }
        child_off[k] = ibuf.size();
        ibuf.insert(ibuf.end(), ch.begin(), ch.end());
    }
    const size_t lds = sizeof(int32_t) * ((size_t)hoff + 4 * (size_t)act_max + 2 * (size_t)R);
    if (lds > 64 * 1024) return fail(RT_ERR_UNSUPPORTED, "rt_dirset_adaptive: level range needs too much LDS");
    auto* set = new rt_dirset();
    set->lmin = lmin;
    set->lmax = lmax;
    set->R = R;
    set->n_origins = n_origins;
    int32_t* d_i = nullptr;
    double* d_d = nullptr;
    hipError_t e = hipGetDevice(&set->dev.device);
    const size_t n = (size_t)std::max<int64_t>(n_origins, 1) * (size_t)R;
    if (e == hipSuccess) e = hipMalloc((void**)&set->dev.dirs, sizeof(double) * 3 * n);
    if (e == hipSuccess) e = hipMalloc((void**)&set->dev.w2, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc((void**)&set->dev_pix, sizeof(int64_t) * n);
    if (e == hipSuccess) e = hipMalloc((void**)&set->dev_level, sizeof(int32_t) * n);
    if (e == hipSuccess) e = hipMalloc((void**)&d_i, sizeof(int32_t) * ibuf.size());
    if (e == hipSuccess) e = hipMalloc((void**)&d_d, sizeof(double) * dbuf.size());
    if (e == hipSuccess) e = hipMemcpyAsync(d_i, ibuf.data(), sizeof(int32_t) * ibuf.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_d, dbuf.data(), sizeof(double) * dbuf.size(), hipMemcpyHostToDevice, s);
    int32_t* ew = error_word();
    if (e == hipSuccess && !ew) e = hipErrorUnknown;
    if (e == hipSuccess) {
        for (int k = 0; k < L; ++k) {
            t.anti[k] = d_i + anti_off[k];
            t.cen[k] = d_d + cen_off[k];
            t.child[k] = k + 1 < L ? d_i + child_off[k] : nullptr;
        }
        if (n_origins > 0) {
            hipLaunchKernelGGL(k_dirset, dim3((unsigned)n_origins), dim3(DS_BLOCK), lds, s, model->pos, model->P,
                               origins_dev, sample_ids_dev, n_sample, t, set->dev_pix, set->dev_level, set->dev.dirs,
                               set->dev.w2, ew);
            e = hipGetLastError();
        }
    }
    // the tables are needed only by this launch
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (d_i) (void)hipFree(d_i);
    if (d_d) (void)hipFree(d_d);
    if (e != hipSuccess) {
        rt_status st = hip_fail(e, "rt_dirset_adaptive");
        rt_dirset_destroy(set);
        return st;
    }
    *out = set;
    return RT_OK;
}

extern "C" rt_status rt_healpix_vec2pix(int32_t nside, const double* dirs, int64_t n, int64_t* pix) {
    if (nside < 1 || (nside & (nside - 1)) || nside > (1 << RT_MAX_LEVEL))
        return rt::fail(RT_ERR_UNSUPPORTED, "rt_healpix_vec2pix: nside must be a power of two up to 2^13");
    if (n < 0 || (n > 0 && (!dirs || !pix))) return rt::fail(RT_ERR_ARG, "rt_healpix_vec2pix: bad arguments");
    for (int64_t i = 0; i < n; ++i) pix[i] = rt::fx_vec2pix(nside, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]);
    return RT_OK;
}
