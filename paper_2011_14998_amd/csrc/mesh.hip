// Re-meshing indicators of an existing model (Section 2.2.2): for a tracer f,
// the relative-change indicator Gf (eq. 6), the local element size L (eq. 8)
// and the desired element size ell (eq. 7) at every point.  One thread per
// point walks its neighbour row; the arithmetic is FP64 in neighbour order.
#include "rt_internal.h"

namespace rt {
namespace {

__global__ __launch_bounds__(256) void k_mesh_indicators(const double* __restrict__ pos,
                                                          const int64_t* __restrict__ off,
                                                          const int32_t* __restrict__ idx, int64_t P,
                                                          const double* __restrict__ f, double f_small,
                                                          double f_large, double G_thres, double* __restrict__ Gf,
                                                          double* __restrict__ L, double* __restrict__ ell) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const double fi = f[i];
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        double g = 0.0, sum = 0.0;
        const int64_t e0 = off[i], e1 = off[i + 1];
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t n = idx[e];
            const double fn = f[n];
            const double r = fabs((fi - fn) / (fi + fn));
            g = r > g ? r : g;
            const double dx = xi - pos[3 * n], dy = yi - pos[3 * n + 1], dz = zi - pos[3 * n + 2];
            sum += sqrt((dx * dx + dy * dy) + dz * dz);
        }
        const double Li = sum / (double)(e1 - e0);
        if (Gf) Gf[i] = g;
        if (L) L[i] = Li;
        if (ell) ell[i] = Li * (g >= G_thres ? f_small : f_large);
    }
}

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" rt_status rt_mesh_indicators(const rt_model* m, const double* f, double f_small, double f_large,
                                        double G_thres, double* Gf, double* L, double* ell, void* stream) {
    if (!m || !f) return fail(RT_ERR_ARG, "rt_mesh_indicators: NULL model or tracer");
    if (m->P == 0) return RT_OK;
    hipLaunchKernelGGL(k_mesh_indicators, dim3(capped_blocks((m->P + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, m->pos, m->off, m->idx, m->P, f, f_small, f_large, G_thres, Gf, L, ell);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
