// Feautrier sweep and J reduction.
//
// Work item = (origin, antipodal pair, 64-frequency chunk); one wavefront per
// item, one frequency per lane.  The line of a pair is
//     reverse(ray -n_r), origin, ray +n_r
// and only u at the origin is needed, so each side is eliminated from its far
// end inwards (second-order Feautrier equation, eq. 1, with second-order
// boundary conditions at both ends) and the two sides meet at the origin.
// Nothing but the running (F, Z) pair and the previous point's optics is kept
// per lane: a line of any length streams through registers.
//
// Rescaled elimination.  With the three-point rows
//     -A_d u_{d-1} + (1 + A_d + C_d) u_d - C_d u_{d+1} = S_d,
//     A_d = 2/(a(a+b)), C_d = 2/(b(a+b)),  a = outer dtau, b = inner dtau,
// and u_d = u_{d+1}/(1+F_d) + Z_d, the recurrences become
//     F_d = b(a+b)/2 + (b/a) F_{d-1}/(1+F_{d-1})
//     Z_d = (b(a+b)/2 S_d + (b/a) Z_{d-1}) / (1 + F_d)
// and at the far end (boundary row from u' = u - I to second order)
//     F_0 = b(1 + b/2),  Z_0 = (b^2/2 S_0 + b I)/(1 + F_0).
// Every term is a sum or quotient of positive numbers, so small optical-depth
// steps lose nothing to cancellation.  At the origin, with h = ab(a+b)/2,
//     u = (h S + b Z_- + a Z_+) / (h + b F_-/(1+F_-) + a F_+/(1+F_+)),
// and with one side empty (dtau t on the other)
//     u = (t^2/2 S + t I + Z) / (t^2/2 + t + F/(1+F)).
//
// Per-point data that is the same for every frequency (point id, ds, the
// velocity projection) is loaded for 64 points at once, one per lane, and
// broadcast with readlane; each lane then gathers its own chi/eta values of
// that point's row -- 64 consecutive values, one coalesced 256-byte read per
// table for FP32.
#include "rt_internal.h"

namespace rt {

namespace {

constexpr int SOLVE_BLOCK = 256;
constexpr int WAVES_PER_BLOCK = SOLVE_BLOCK / 64;

__device__ inline double readlane_d(double v, int j) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_readlane(p.x, j);
    p.y = __builtin_amdgcn_readlane(p.y, j);
    return __builtin_bit_cast(double, p);
}

__device__ inline int readlane_i(int v, int j) { return __builtin_amdgcn_readlane(v, j); }

struct LaneFreq {
    int f;       // global frequency index of this lane (clamped to F-1 when inactive)
    bool active;
    int fb;      // start of the lane's block
    int L;       // length of the block
    int fl;      // index inside the block
    double inv_dx;
};

__device__ inline LaneFreq lane_freq(const SolveLaunch& a, int fc, int lane) {
    LaneFreq lf;
    int f = fc * 64 + lane;
    lf.active = f < a.F;
    lf.f = lf.active ? f : a.F - 1;
    int b = 0;
#pragma unroll
    for (int bb = 1; bb < RT_MAX_FREQ_BLOCKS; ++bb)
        if (bb < a.n_blocks && lf.f >= a.blk_start[bb]) b = bb;
    int fb = a.blk_start[0], nb = a.blk_start[1];
    double idx = a.inv_dx[0];
#pragma unroll
    for (int bb = 1; bb < RT_MAX_FREQ_BLOCKS; ++bb)
        if (bb == b) {
            fb = a.blk_start[bb];
            nb = a.blk_start[bb + 1];
            idx = a.inv_dx[bb];
        }
    lf.fb = fb;
    lf.L = nb - fb;
    lf.fl = lf.f - fb;
    lf.inv_dx = idx;
    return lf;
}

// One row of the rescaled elimination (see the file header).
template <typename T>
__device__ inline void row_update(bool far_end, T a, T b, T S, T I, T& F, T& Z) {
    if (far_end) {
        F = b * ((T)1 + (T)0.5 * b);
        Z = ((T)0.5 * b * b * S + b * I) / ((T)1 + F);
    } else {
        T hb = (T)0.5 * b * (a + b);
        T ba = b / a;
        T Fn = hb + ba * (F / ((T)1 + F));
        Z = (hb * S + ba * Z) / ((T)1 + Fn);
        F = Fn;
    }
}

template <typename T>
__device__ inline void row_update_policy(bool far_end, T a, T b, T S, T I, T& F, T& Z, double thr) {
    row_update<T>(far_end, a, b, S, I, F, Z);
}

// FP32 sweep: rows whose optical-depth steps fall below the threshold are
// eliminated in FP64 (the coefficients b(a+b)/2 and b/a lose relative
// accuracy to rounding of the tiny steps first).
template <>
__device__ inline void row_update_policy<float>(bool far_end, float a, float b, float S, float I, float& F,
                                                float& Z, double thr) {
    float m = far_end ? b : fminf(a, b);
    if ((double)m < thr) {
        double Fd = F, Zd = Z;
        row_update<double>(far_end, (double)a, (double)b, (double)S, (double)I, Fd, Zd);
        F = (float)Fd;
        Z = (float)Zd;
    } else {
        row_update<float>(far_end, a, b, S, I, F, Z);
    }
}

template <typename T>
__device__ inline T origin_u(int64_t nm, int64_t np, T a, T b, T Fm, T Zm, T Fp, T Zp, T S, T I) {
    if (nm > 0 && np > 0) {
        T h = (T)0.5 * a * b * (a + b);
        return (h * S + b * Zm + a * Zp) / (h + b * (Fm / ((T)1 + Fm)) + a * (Fp / ((T)1 + Fp)));
    }
    if (np > 0) {
        T h = (T)0.5 * b * b;
        return (h * S + b * I + Zp) / (h + b + Fp / ((T)1 + Fp));
    }
    if (nm > 0) {
        T h = (T)0.5 * a * a;
        return (h * S + a * I + Zm) / (h + a + Fm / ((T)1 + Fm));
    }
    return I;
}

template <typename T>
__device__ inline T origin_u_policy(int64_t nm, int64_t np, T a, T b, T Fm, T Zm, T Fp, T Zp, T S, T I,
                                    double thr) {
    return origin_u<T>(nm, np, a, b, Fm, Zm, Fp, Zp, S, I);
}

template <>
__device__ inline float origin_u_policy<float>(int64_t nm, int64_t np, float a, float b, float Fm, float Zm,
                                               float Fp, float Zp, float S, float I, double thr) {
    float m = (nm > 0 && np > 0) ? fminf(a, b) : (np > 0 ? b : a);
    if ((nm > 0 || np > 0) && (double)m < thr)
        return (float)origin_u<double>(nm, np, a, b, Fm, Zm, Fp, Zp, S, I);
    return origin_u<float>(nm, np, a, b, Fm, Zm, Fp, Zp, S, I);
}

struct Side {
    int64_t base;
    int64_t n;
};

// Eliminate one side of the line, far end first, up to the origin.
template <typename T, bool MOVING>
__device__ inline void sweep(const SolveLaunch& a, const T* __restrict__ chi, const T* __restrict__ eta,
                             const Side sd, const LaneFreq& lf, int lane, double nx, double ny, double nz,
                             float vox, float voy, float voz, T chi_o, T I, T& Fs, T& Zs, T& dt_last) {
    const int32_t* __restrict__ ids = a.ray_ids;
    const double* __restrict__ Zr = a.ray_Z;
    const int64_t ld = a.ld;
    T c_prev = (T)0, S_prev = (T)0, dt_out = (T)0;
    double ds_prev = 0.0;
    int64_t done = 0;
    for (int64_t hi = sd.n - 1; hi >= 0; hi -= 64) {
        const int cnt = (int)(hi + 1 < 64 ? hi + 1 : 64);
        const int64_t e = hi - lane;
        const bool v = lane < cnt;
        int q_l = 0;
        double ds_l = 0.0, dot_l = 0.0;
        if (v) {
            q_l = ids[sd.base + e];
            double z = Zr[sd.base + e];
            double zi = e > 0 ? Zr[sd.base + e - 1] : 0.0;
            ds_l = z - zi;
            if (MOVING) {
                const float* vq = a.vel + 3 * (int64_t)q_l;
                double dvx = (double)vq[0] - (double)vox;
                double dvy = (double)vq[1] - (double)voy;
                double dvz = (double)vq[2] - (double)voz;
                dot_l = (nx * dvx + ny * dvy) + nz * dvz;
            }
        }
        for (int j = 0; j < cnt; ++j) {
            const int q = readlane_i(q_l, j);
            const double ds = readlane_d(ds_l, j);
            const T* cr = chi + (int64_t)q * ld;
            const T* er = eta + (int64_t)q * ld;
            T c, et;
            if (MOVING) {
                const double dot = readlane_d(dot_l, j);
                const double delta = dot * lf.inv_dx;
                const double kf = floor(delta);
                const T t = (T)(delta - kf);
                const int k = (int)kf;
                int ia = lf.fl - k, ib = lf.fl - k - 1;
                ia = ia < 0 ? 0 : (ia > lf.L - 1 ? lf.L - 1 : ia);
                ib = ib < 0 ? 0 : (ib > lf.L - 1 ? lf.L - 1 : ib);
                const T ca = cr[lf.fb + ia], cb = cr[lf.fb + ib];
                const T ea = er[lf.fb + ia], eb = er[lf.fb + ib];
                c = ((T)1 - t) * ca + t * cb;
                et = ((T)1 - t) * ea + t * eb;
            } else {
                c = cr[lf.f];
                et = er[lf.f];
            }
            const T S = et / c;
            if (done > 0) {
                const T dt = ((T)0.5 * (c_prev + c)) * (T)ds_prev;
                row_update_policy<T>(done == 1, dt_out, dt, S_prev, I, Fs, Zs, a.dtau_fp64_below);
                dt_out = dt;
            }
            c_prev = c;
            S_prev = S;
            ds_prev = ds;
            ++done;
        }
    }
    if (sd.n > 0) {
        const T dt = ((T)0.5 * (c_prev + chi_o)) * (T)ds_prev;
        row_update_policy<T>(sd.n == 1, dt_out, dt, S_prev, I, Fs, Zs, a.dtau_fp64_below);
        dt_last = dt;
    }
}

template <typename T, bool MOVING>
__device__ inline void solve_item(const SolveLaunch& a, int64_t w, int nfc, int lane) {
    const T* __restrict__ chi = (const T*)a.chi;
    const T* __restrict__ eta = (const T*)a.eta;
    const int fc = (int)(w % nfc);
    const int64_t pr = w / nfc;
    const int64_t r = pr % a.R;
    const int64_t oi = pr / a.R;
    const LaneFreq lf = lane_freq(a, fc, lane);
    const int64_t o = a.origins ? (int64_t)a.origins[oi] : oi;
    if (o < 0 || o >= a.P) {
        if (lane == 0) atomicOr(a.err, ERRBIT_ORIGIN);
        return;
    }
    const int64_t slot_p = oi * 2 * a.R + 2 * r;
    Side sp, sm;
    sp.base = a.ray_off[slot_p];
    sp.n = a.ray_off[slot_p + 1] - sp.base;
    sm.base = a.ray_off[slot_p + 1];
    sm.n = a.ray_off[slot_p + 2] - sm.base;
    const double* dv = a.dirs + 3 * ((a.per_origin ? oi * a.R : 0) + r);
    const double nx = dv[0], ny = dv[1], nz = dv[2];
    float vox = 0.f, voy = 0.f, voz = 0.f;
    if (MOVING) {
        vox = a.vel[3 * o];
        voy = a.vel[3 * o + 1];
        voz = a.vel[3 * o + 2];
    }
    const T I = (T)a.I_bc[lf.f];
    const T chi_o = chi[o * a.ld + lf.f];
    const T S_o = eta[o * a.ld + lf.f] / chi_o;
    T Fm = 0, Zm = 0, dm = 0, Fp = 0, Zp = 0, dp = 0;
    sweep<T, MOVING>(a, chi, eta, sm, lf, lane, nx, ny, nz, vox, voy, voz, chi_o, I, Fm, Zm, dm);
    sweep<T, MOVING>(a, chi, eta, sp, lf, lane, nx, ny, nz, vox, voy, voz, chi_o, I, Fp, Zp, dp);
    const T u = origin_u_policy<T>(sm.n, sp.n, dm, dp, Fm, Zm, Fp, Zp, S_o, I, a.dtau_fp64_below);
    if (lf.active) {
        ((T*)a.u)[(oi * a.R + r) * a.F + lf.f] = u;
        if (!(u == u) || u - u != (T)0) atomicOr(a.err, ERRBIT_NONFINITE);
    }
}

template <typename T, bool MOVING>
__global__ __launch_bounds__(SOLVE_BLOCK) void k_solve_direct(const SolveLaunch a) {
    const int lane = threadIdx.x & 63;
    const int nfc = (a.F + 63) / 64;
    const int64_t n_items = a.n_origins * a.R * nfc;
    const int64_t it = (int64_t)blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (it >= n_items) return;
    const int64_t w = a.items ? (int64_t)a.items[it] : it;
    solve_item<T, MOVING>(a, w, nfc, lane);
}

// Persistent variant: a fixed grid of waves drains the item queue; each wave
// takes the next item with one atomic and exits when the queue is empty, so
// every wave reaches the end.
template <typename T, bool MOVING>
__global__ __launch_bounds__(SOLVE_BLOCK) void k_solve_persist(const SolveLaunch a) {
    const int lane = threadIdx.x & 63;
    const int nfc = (a.F + 63) / 64;
    const int64_t n_items = a.n_origins * a.R * nfc;
    for (;;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(a.queue, 1);
        it = __builtin_amdgcn_readfirstlane(it);
        if ((int64_t)it >= n_items) break;
        const int64_t w = a.items ? (int64_t)a.items[it] : (int64_t)it;
        solve_item<T, MOVING>(a, w, nfc, lane);
    }
}

// J[o][f] = sum over pairs, ascending, of w2_r u_r[f] (eq. 3, eq. 4).
template <typename T>
__global__ __launch_bounds__(256) void k_reduce(const SolveLaunch a) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n_origins * a.F) return;
    const int64_t oi = i / a.F;
    const int f = (int)(i - oi * a.F);
    const T* __restrict__ u = (const T*)a.u + oi * a.R * a.F + f;
    const double* __restrict__ w2 = a.w2 + (a.per_origin ? oi * a.R : 0);
    T acc = (T)0;
    for (int64_t r = 0; r < a.R; ++r) acc += (T)w2[r] * u[r * a.F];
    ((T*)a.J)[i] = acc;
}

// ---------------------------------------------------------------- length binning
// Bin b holds pairs whose line length N = n_- + n_+ + 1 has floor(4 log2 N) = b
// (quarter-octave bins, the last bin open-ended).  Items are laid out bin by
// bin, longest lines first, so the persistent grid starts the long lines early
// and finishes on short ones.
__device__ inline int bin_of(int64_t N, int n_bins) {
    int b = 0;
    double x = (double)N;
    b = (int)floor(4.0 * log2(x));
    if (b < 0) b = 0;
    if (b > n_bins - 1) b = n_bins - 1;
    return b;
}

__global__ __launch_bounds__(256) void k_bin_count(const SolveLaunch a) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= a.n_origins * a.R) return;
    const int64_t s = 2 * p;  // slot of the +ray: origin*2R + 2r = 2*(origin*R + r)
    const int64_t N = a.ray_off[s + 2] - a.ray_off[s] + 1;
    atomicAdd(&a.bin_counts[bin_of(N, a.n_bins)], 1);
}

__global__ void k_bin_offsets(const SolveLaunch a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int run = 0;
    for (int b = a.n_bins - 1; b >= 0; --b) {
        int c = a.bin_counts[b];
        a.bin_cursor[b] = run;
        run += c;
    }
}

__global__ __launch_bounds__(256) void k_bin_scatter(const SolveLaunch a, int32_t* __restrict__ items) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= a.n_origins * a.R) return;
    const int64_t s = 2 * p;
    const int64_t N = a.ray_off[s + 2] - a.ray_off[s] + 1;
    const int nfc = (a.F + 63) / 64;
    const int pos = atomicAdd(&a.bin_cursor[bin_of(N, a.n_bins)], 1);
    for (int c = 0; c < nfc; ++c) items[(int64_t)pos * nfc + c] = (int32_t)(p * nfc + c);
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int64_t solve_items(const SolveLaunch& a) { return a.n_origins * a.R * ((a.F + 63) / 64); }

size_t bin_workspace(int64_t n_items, int32_t n_bins) {
    return (size_t)n_items * sizeof(int32_t) + (size_t)(2 * n_bins + 2) * sizeof(int32_t) + 256;
}

hipError_t launch_bin(const SolveLaunch& a0, void* ws, int32_t** items_out, hipStream_t s) {
    SolveLaunch a = a0;
    const int64_t n_items = solve_items(a);
    int32_t* items = (int32_t*)ws;
    int32_t* counts = items + ((n_items + 63) / 64) * 64;
    a.bin_counts = counts;
    a.bin_cursor = counts + a.n_bins + 1;
    hipError_t e = launch_fill_i32(counts, a.n_bins + 1, 0, s);
    if (e != hipSuccess) return e;
    const int64_t pairs = a.n_origins * a.R;
    if (pairs > 0) {
        hipLaunchKernelGGL(k_bin_count, dim3(nblocks(pairs, 256)), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_bin_offsets, dim3(1), dim3(64), 0, s, a);
        hipLaunchKernelGGL(k_bin_scatter, dim3(nblocks(pairs, 256)), dim3(256), 0, s, a, items);
    }
    *items_out = items;
    return hipGetLastError();
}

hipError_t launch_solve(const SolveLaunch& a, int precision, hipStream_t s) {
    const int64_t n_items = solve_items(a);
    if (n_items == 0) return hipSuccess;
    const bool moving = a.vel != nullptr;
    if (a.schedule == RT_SCHED_BINNED) {
        dim3 grid((unsigned)((a.grid_waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK));
        if (precision == RT_F64) {
            if (moving) hipLaunchKernelGGL((k_solve_persist<double, true>), grid, dim3(SOLVE_BLOCK), 0, s, a);
            else hipLaunchKernelGGL((k_solve_persist<double, false>), grid, dim3(SOLVE_BLOCK), 0, s, a);
        } else {
            if (moving) hipLaunchKernelGGL((k_solve_persist<float, true>), grid, dim3(SOLVE_BLOCK), 0, s, a);
            else hipLaunchKernelGGL((k_solve_persist<float, false>), grid, dim3(SOLVE_BLOCK), 0, s, a);
        }
    } else {
        dim3 grid(nblocks(n_items, WAVES_PER_BLOCK));
        if (precision == RT_F64) {
            if (moving) hipLaunchKernelGGL((k_solve_direct<double, true>), grid, dim3(SOLVE_BLOCK), 0, s, a);
            else hipLaunchKernelGGL((k_solve_direct<double, false>), grid, dim3(SOLVE_BLOCK), 0, s, a);
        } else {
            if (moving) hipLaunchKernelGGL((k_solve_direct<float, true>), grid, dim3(SOLVE_BLOCK), 0, s, a);
            else hipLaunchKernelGGL((k_solve_direct<float, false>), grid, dim3(SOLVE_BLOCK), 0, s, a);
        }
    }
    return hipGetLastError();
}

hipError_t launch_reduce(const SolveLaunch& a, int precision, hipStream_t s) {
    const int64_t n = a.n_origins * a.F;
    if (n == 0) return hipSuccess;
    if (precision == RT_F64)
        hipLaunchKernelGGL(k_reduce<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_reduce<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace rt
