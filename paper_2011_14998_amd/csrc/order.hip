// Per-pair sweep orders.
//
// The sweep's work item (origin, pair r) runs along the line through the origin
// in direction d_r.  Items of one pair whose origins sit on nearly the same line
// read nearly the same points, so when they run at the same time the chi and
// eta rows they read are served by L2.  For each pair of a uniform direction
// set the origin positions are sorted by a key of three parts: the origin's
// segment (model of a batch), the 2D Morton code of its position projected on
// two axes across d_r, and its position along d_r (16 bits each over the
// segment's bounding sphere).  One radix sort per pair (hipCUB) on the device.
// The order only decides which items run together; every item's result is the
// same in any order.
#include <hipcub/hipcub.hpp>

#include "rt_internal.h"

namespace rt {

namespace {

__device__ inline uint32_t spread16(uint32_t v) {  // 16 bits -> the even bits of 32
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ inline uint32_t quant16(double x, double lo, double inv_w) {
    const double q = (x - lo) * inv_w;
    return q <= 0.0 ? 0u : (q >= 65535.0 ? 65535u : (uint32_t)q);
}

// keys[k], vals[k] = k for origin position k and pair direction d
__global__ __launch_bounds__(256) void k_pair_keys(const double* __restrict__ pos, const int32_t* __restrict__ origins,
                                                    int64_t n_o, int64_t P, double dx, double dy, double dz,
                                                    const OrderSeg* __restrict__ segs, int n_seg,
                                                    uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n_o) return;
    int64_t o = origins ? (int64_t)origins[k] : k;
    if (o < 0 || o >= P) o = 0;  // invalid ids are reported by the walk; any key will do
    // the segment holding position k: the first whose end is beyond k
    int lo = 0, hi = n_seg - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (segs[mid].end > k) hi = mid;
        else lo = mid + 1;
    }
    const OrderSeg g = segs[lo];
    // two unit axes across d: u = (a x d)/|a x d| with a the x axis (the y axis when d is
    // near x), v = d x u
    double ax = 1.0, ay = 0.0;
    if (fabs(dx) >= 0.9) {
        ax = 0.0;
        ay = 1.0;
    }
    double ux = ay * dz, uy = -ax * dz, uz = ax * dy - ay * dx;
    const double un = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
    ux *= un;
    uy *= un;
    uz *= un;
    const double vx = dy * uz - dz * uy, vy = dz * ux - dx * uz, vz = dx * uy - dy * ux;
    const double px = pos[3 * o], py = pos[3 * o + 1], pz = pos[3 * o + 2];
    const double inv_w = g.rho > 0.0 ? 65536.0 / (2.0 * g.rho) : 0.0;
    const uint32_t qu = quant16(px * ux + py * uy + pz * uz, g.c[0] * ux + g.c[1] * uy + g.c[2] * uz - g.rho, inv_w);
    const uint32_t qv = quant16(px * vx + py * vy + pz * vz, g.c[0] * vx + g.c[1] * vy + g.c[2] * vz - g.rho, inv_w);
    const uint32_t qd = quant16(px * dx + py * dy + pz * dz, g.c[0] * dx + g.c[1] * dy + g.c[2] * dz - g.rho, inv_w);
    keys[k] = ((uint64_t)lo << 48) | ((uint64_t)(spread16(qu) | (spread16(qv) << 1)) << 16) | qd;
    vals[k] = (int32_t)k;
}

size_t sort_temp_bytes(int64_t n_o) {
    size_t tb = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                             (const int32_t*)nullptr, (int32_t*)nullptr, (int)n_o, 0, 64);
    return tb;
}

inline size_t al256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

size_t pair_order_workspace(int64_t n_o) {
    return 2 * al256(sizeof(uint64_t) * (size_t)n_o) + al256(sizeof(int32_t) * (size_t)n_o) +
           al256(sort_temp_bytes(n_o));
}

hipError_t build_pair_orders(const double* pos, int64_t P, const int32_t* origins, int64_t n_o, const double* dirs_host,
                             int64_t R, const OrderSeg* segs, int n_seg, int32_t* out, void* ws, hipStream_t s) {
    if (n_o <= 0 || R <= 0) return hipSuccess;
    if (n_o > INT32_MAX || n_seg <= 0 || n_seg > 65535) return hipErrorInvalidValue;
    char* w = (char*)ws;
    uint64_t* kin = (uint64_t*)w;
    w += al256(sizeof(uint64_t) * (size_t)n_o);
    uint64_t* kout = (uint64_t*)w;
    w += al256(sizeof(uint64_t) * (size_t)n_o);
    int32_t* vin = (int32_t*)w;
    w += al256(sizeof(int32_t) * (size_t)n_o);
    size_t tb = sort_temp_bytes(n_o);
    const unsigned g = (unsigned)((n_o + 255) / 256);
    for (int64_t r = 0; r < R; ++r) {
        const double* d = dirs_host + 3 * r;
        hipLaunchKernelGGL(k_pair_keys, dim3(g), dim3(256), 0, s, pos, origins, n_o, P, d[0], d[1], d[2], segs, n_seg,
                           kin, vin);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipcub::DeviceRadixSort::SortPairs((void*)w, tb, kin, kout, vin, out + r * n_o, (int)n_o, 0, 64, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rt
