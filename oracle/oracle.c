/*
 * CPU oracle for the adaptive ray-tracing radiative-transfer hot path
 * (De Ceuster et al., "Magritte II", arXiv 2011.14998).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * FP64 reference that the HIP library is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant generator with the HIP
 * library.
 *
 * Build: gcc -O2 -std=gnu11 -ffp-contract=off -fno-fast-math -fno-builtin-sin
 *        -fno-builtin-cos -fopenmp -shared -fPIC
 * No FMA contraction, no fast-math: every floating-point operation below is a
 * single IEEE-754 double operation, evaluated in the order written.
 *
 * What is computed, step by step, with the passage each step follows:
 *   HEALPix ring-scheme pixel centres and pixel lookup, 12*4^l pixels of equal
 *       area at level l (Section 2.1.3; Gorski et al. 2005 for the scheme).
 *   Uniform direction set: antipodal pairs of level-l pixels (Section 2.1.3:
 *       rays come in antipodal pairs), weight w = 1/(12*4^l) per ray (eq. 4).
 *   Adaptive direction set (Section 2.1.3, Fig. 1): per origin, histogram the
 *       directions to a sample of points at l_max, downgrade through the
 *       hierarchy, refine the top half of the pairs per level.
 *   Ray tracing (Section 2.1, Fig. 2): step from point to point along a
 *       straight line; each step goes to the forward neighbour closest to the
 *       ray axis; the distance increment is the projection of the edge.
 *   Line assembly, Doppler-shifted optics, optical depth (Section 2.1.1 for the
 *       velocity, eq. 1 for S and tau).
 *   Second-order Feautrier equation (eq. 1) with second-order boundary
 *       conditions (Section 2.1), solved for u at the origin by a two-sided
 *       rescaled elimination.
 *   Mean intensity J = sum over rays of w*u (eq. 3, eq. 4).
 *
 * Readings of what the paper leaves unstated are documented next to each step
 * (boundary intensity, quadrature of tau, elimination form, tie rules).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ HEALPix */

static int64_t isqrt64(int64_t v) {
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

OR_API int64_t or_hp_npix(int64_t nside) { return 12 * nside * nside; }

/* Ring index (1 .. 4*nside-1) of pixel p, and the z/phi of its centre. */
static void hp_ring_centre(int64_t nside, int64_t p, int64_t* ring, double* z, double* phi) {
    const int64_t npix = 12 * nside * nside;
    const int64_t ncap = 2 * nside * (nside - 1);
    if (p < ncap) {                       /* north polar cap */
        int64_t i = (1 + isqrt64(1 + 2 * p)) >> 1;
        int64_t j = p + 1 - 2 * i * (i - 1); /* 1 .. 4i */
        *ring = i;
        *z = 1.0 - (double)(i * i) / (double)(3 * nside * nside);
        *phi = (double)(2 * j - 1) * M_PI / (double)(4 * i);
    } else if (p < npix - ncap) {         /* equatorial belt */
        int64_t q = p - ncap;
        int64_t i = q / (4 * nside) + nside;
        int64_t k = q % (4 * nside);      /* 0 .. 4nside-1 */
        int64_t s = (i - nside + 1) & 1;
        *ring = i;
        *z = (double)(2 * (2 * nside - i)) / (double)(3 * nside);
        *phi = (double)(2 * k + s) * M_PI / (double)(4 * nside);
    } else {                              /* south polar cap */
        int64_t q = npix - p;
        int64_t i = (1 + isqrt64(2 * q - 1)) >> 1;
        int64_t j = 4 * i + 1 - (q - 2 * i * (i - 1));
        *ring = 4 * nside - i;
        *z = -(1.0 - (double)(i * i) / (double)(3 * nside * nside));
        *phi = (double)(2 * j - 1) * M_PI / (double)(4 * i);
    }
}

/* Unit vector of the centre of ring-scheme pixel p at resolution nside.
 * sin and cos are called separately (the build keeps the compiler from
 * fusing them into sincos, which may round differently). */
OR_API void or_hp_pix2vec(int64_t nside, int64_t p, double* v) {
    int64_t ring;
    double z, phi;
    hp_ring_centre(nside, p, &ring, &z, &phi);
    double st = sqrt((1.0 - z) * (1.0 + z));
    v[0] = st * cos(phi);
    v[1] = st * sin(phi);
    v[2] = z;
}

OR_API int64_t or_hp_ring_of(int64_t nside, int64_t p) {
    int64_t ring;
    double z, phi;
    hp_ring_centre(nside, p, &ring, &z, &phi);
    return ring;
}

/* Pixel lookup from (z, phi), phi in [0, 2 pi). */
static int64_t hp_zphi2pix(int64_t nside, double z, double phi) {
    const int64_t npix = 12 * nside * nside;
    const int64_t ncap = 2 * nside * (nside - 1);
    double za = fabs(z);
    double tt = phi / (0.5 * M_PI);       /* [0, 4) */
    if (tt >= 4.0) tt = 0.0;
    if (za <= 2.0 / 3.0) {
        double t1 = (double)nside * (0.5 + tt);
        double t2 = (double)nside * z * 0.75;
        int64_t jp = (int64_t)floor(t1 - t2);
        int64_t jm = (int64_t)floor(t1 + t2);
        int64_t ir = nside + 1 + jp - jm;          /* 1 .. 2nside+1 */
        int64_t kshift = 1 - (ir & 1);
        int64_t ip = (jp + jm - nside + kshift + 1) / 2;
        ip = ((ip % (4 * nside)) + 4 * nside) % (4 * nside);
        return ncap + (ir - 1) * 4 * nside + ip;
    } else {
        double tp = tt - floor(tt);
        double tmp = (double)nside * sqrt(3.0 * (1.0 - za));
        int64_t jp = (int64_t)floor(tp * tmp);
        int64_t jm = (int64_t)floor((1.0 - tp) * tmp);
        int64_t ir = jp + jm + 1;
        int64_t ip = (int64_t)floor(tt * (double)ir);
        ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
        if (z > 0.0) return 2 * ir * (ir - 1) + ip;
        return npix - 2 * ir * (ir + 1) + ip;
    }
}

/* Pixel containing the direction of v (need not be normalised; v != 0).
 * Uses the C library's atan2 for the azimuth. */
OR_API int64_t or_hp_vec2pix(int64_t nside, const double* v) {
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double z = v[2] / r;
    double phi = atan2(v[1], v[0]);
    if (phi < 0.0) phi += 2.0 * M_PI;
    return hp_zphi2pix(nside, z, phi);
}

/* Antipodal pixel: the pixel containing minus the centre of p. */
static int64_t hp_antipode(int64_t nside, int64_t p) {
    double v[3];
    or_hp_pix2vec(nside, p, v);
    v[0] = -v[0]; v[1] = -v[1]; v[2] = -v[2];
    return or_hp_vec2pix(nside, v);
}

OR_API int64_t or_hp_antipode(int64_t nside, int64_t p) { return hp_antipode(nside, p); }

/* Parent at nside/2 in the nested hierarchy: the coarse pixel containing the
 * centre of p (each coarse pixel is the union of its 4 children). */
OR_API int64_t or_hp_parent(int64_t nside, int64_t p) {
    double v[3];
    or_hp_pix2vec(nside, p, v);
    return or_hp_vec2pix(nside / 2, v);
}

/* ---------------------------------------------------------- direction sets */

/* Uniform set at resolution nside: every antipodal pair of pixels once, the
 * member with the smaller ring-scheme index being canonical; pairs ascending
 * in that index.  Ray direction of pair r is the centre of its canonical
 * pixel; the partner ray is its exact negation.  w2[r] = 2 w, w = 1/(12 nside^2)
 * (eq. 4, the pair carries both rays).  Returns the number of pairs. */
OR_API int64_t or_dirset_uniform(int64_t nside, int64_t* pix, double* dirs, double* w2) {
    int64_t npix = 12 * nside * nside, R = 0;
    for (int64_t p = 0; p < npix; ++p) {
        if (hp_antipode(nside, p) <= p) continue;
        if (pix) pix[R] = p;
        if (dirs) or_hp_pix2vec(nside, p, dirs + 3 * R);
        if (w2) w2[R] = 2.0 / (double)npix;
        ++R;
    }
    return R;
}

/* ------------------------------------------- pixel lookup for adaptive sets
 *
 * The adaptive direction set classifies the directions to sample points into
 * pixels, so CPU and GPU must classify boundary directions identically.  The
 * lookup therefore uses a square root and an arctangent built only from IEEE
 * +, -, *, / in a fixed order (no library transcendental), evaluated
 * identically by the HIP library:
 *   fx_sqrt(x):    seed from the exponent bits (bits/2 + bias), then six
 *                  Newton steps y <- 0.5 (y + x / y).
 *   fx_atan2(y,x): reduce to t = min/max in [0,1]; if t > tan(pi/8), use
 *                  t' = (t - 1)/(t + 1) and add pi/4; atan(t') by its Taylor
 *                  series to t'^43 (Horner in t'^2, coefficient (-1)^k/(2k+1)
 *                  formed by one division); then undo the octant.
 * Both agree with the C library to a few ulp (pinned by the tests). */
static double fx_sqrt(double x) {
    if (!(x > 0.0)) return 0.0;
    union { double d; uint64_t u; } b;
    b.d = x;
    b.u = (b.u >> 1) + 0x1FF8000000000000ULL;
    double y = b.d;
    for (int i = 0; i < 6; ++i) y = 0.5 * (y + x / y);
    return y;
}

static double fx_atan2(double y, double x) {
    double ax = fabs(x), ay = fabs(y);
    if (ax == 0.0 && ay == 0.0) return 0.0;
    int swap = ay > ax;
    double mx = swap ? ay : ax, mn = swap ? ax : ay;
    double t = mn / mx, base = 0.0;
    if (t > 0.41421356237309503) {
        t = (t - 1.0) / (t + 1.0);
        base = 0.78539816339744831;
    }
    double t2 = t * t, p = 0.0;
    for (int k = 21; k >= 0; --k) {
        double c = (k & 1 ? -1.0 : 1.0) / (double)(2 * k + 1);
        p = p * t2 + c;
    }
    double r = base + t * p;
    if (swap) r = 1.5707963267948966 - r;
    if (x < 0.0) r = 3.1415926535897931 - r;
    if (y < 0.0) r = -r;
    return r;
}

/* Pixel of the direction of (vx, vy, vz) with the fixed-arithmetic lookup. */
static int64_t fx_vec2pix(int64_t nside, double vx, double vy, double vz) {
    const int64_t npix = 12 * nside * nside;
    const int64_t ncap = 2 * nside * (nside - 1);
    double r = fx_sqrt((vx * vx + vy * vy) + vz * vz);
    double z = vz / r;
    double phi = fx_atan2(vy, vx);
    if (phi < 0.0) phi = phi + 6.2831853071795862;
    double za = fabs(z);
    double tt = phi / 1.5707963267948966;
    if (tt >= 4.0) tt = 0.0;
    if (za <= 2.0 / 3.0) {
        double t1 = (double)nside * (0.5 + tt);
        double t2 = (double)nside * z * 0.75;
        int64_t jp = (int64_t)floor(t1 - t2);
        int64_t jm = (int64_t)floor(t1 + t2);
        int64_t ir = nside + 1 + jp - jm;
        int64_t kshift = 1 - (ir & 1);
        int64_t ip = (jp + jm - nside + kshift + 1) / 2;
        ip = ((ip % (4 * nside)) + 4 * nside) % (4 * nside);
        return ncap + (ir - 1) * 4 * nside + ip;
    } else {
        double tp = tt - floor(tt);
        double tmp = (double)nside * fx_sqrt(3.0 * (1.0 - za));
        int64_t jp = (int64_t)floor(tp * tmp);
        int64_t jm = (int64_t)floor((1.0 - tp) * tmp);
        int64_t ir = jp + jm + 1;
        int64_t ip = (int64_t)floor(tt * (double)ir);
        ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
        if (z > 0.0) return 2 * ir * (ir - 1) + ip;
        return npix - 2 * ir * (ir + 1) + ip;
    }
}

OR_API double or_fx_sqrt(double x) { return fx_sqrt(x); }
OR_API double or_fx_atan2(double y, double x) { return fx_atan2(y, x); }
OR_API int64_t or_fx_vec2pix(int64_t nside, const double* v) { return fx_vec2pix(nside, v[0], v[1], v[2]); }

/* --------------------------------------------------- adaptive direction sets */

typedef struct { int64_t cnt; int64_t pix; } or_key;

static int key_cmp(const void* a, const void* b) {
    const or_key* x = (const or_key*)a;
    const or_key* y = (const or_key*)b;
    if (x->cnt != y->cnt) return x->cnt > y->cnt ? -1 : 1;   /* count descending */
    return x->pix < y->pix ? -1 : (x->pix > y->pix ? 1 : 0); /* then ring index ascending */
}

typedef struct { int32_t level; int64_t pix; } or_leaf;

static int leaf_cmp(const void* a, const void* b) {
    const or_leaf* x = (const or_leaf*)a;
    const or_leaf* y = (const or_leaf*)b;
    if (x->level != y->level) return x->level < y->level ? -1 : 1;
    return x->pix < y->pix ? -1 : (x->pix > y->pix ? 1 : 0);
}

/* Number of pairs per origin of the adaptive set (lmin, lmax). */
OR_API int64_t or_dirset_adaptive_R(int32_t lmin, int32_t lmax) {
    int64_t R = 0, act = 6LL << (2 * lmin);
    for (int32_t l = lmin; l < lmax; ++l) {
        R += act / 2;
        act = 4 * (act / 2);
    }
    return R + act;
}

/* Adaptive direction set per origin (Section 2.1.3, Fig. 1).
 * For origin i: every sample point s != i with x_s != x_i adds one to the
 * level-lmax pixel containing x_s - x_i (fixed-arithmetic lookup above).  The
 * pixel histogram is downgraded to every coarser level by summing the four
 * children of each pixel (the nested hierarchy).  The count of an antipodal
 * pair is the sum over both of its pixels.  Starting from every pair at lmin,
 * at each level the active pairs are ranked by count (descending, ties to the
 * smaller canonical index) and the first half is refined into the pairs of
 * their children; the rest become leaves at that level; all active pairs at
 * lmax are leaves.  Leaves are written ordered by (level, canonical index):
 * pix, level, direction (centre of the canonical pixel at its level) and pair
 * weight 2/(12*4^level).  Returns R (pairs per origin). */
OR_API int64_t or_dirset_adaptive(const double* pos, int64_t P, const int32_t* origins, int64_t n_origins,
                                  const int32_t* sample, int64_t n_sample, int32_t lmin, int32_t lmax,
                                  int64_t* pix_out, int32_t* level_out, double* dirs_out, double* w2_out,
                                  int nthreads) {
    const int64_t R = or_dirset_adaptive_R(lmin, lmax);
    const int32_t L = lmax - lmin + 1;
    int64_t* npix = (int64_t*)malloc(sizeof(int64_t) * L);
    int64_t** anti = (int64_t**)malloc(sizeof(int64_t*) * L);
    int64_t** par = (int64_t**)malloc(sizeof(int64_t*) * L);
    for (int32_t k = 0; k < L; ++k) {
        int64_t ns = 1LL << (lmin + k);
        npix[k] = 12 * ns * ns;
        anti[k] = (int64_t*)malloc(sizeof(int64_t) * npix[k]);
        par[k] = (int64_t*)malloc(sizeof(int64_t) * npix[k]);
        for (int64_t p = 0; p < npix[k]; ++p) {
            anti[k][p] = hp_antipode(ns, p);
            par[k][p] = k > 0 ? or_hp_parent(ns, p) : -1;
        }
    }
    (void)P;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t oi = 0; oi < n_origins; ++oi) {
        const int64_t o = origins[oi];
        int64_t** h = (int64_t**)malloc(sizeof(int64_t*) * L);
        for (int32_t k = 0; k < L; ++k) h[k] = (int64_t*)calloc((size_t)npix[k], sizeof(int64_t));
        const int64_t nsm = 1LL << lmax;
        for (int64_t j = 0; j < n_sample; ++j) {
            const int64_t s = sample[j];
            if (s == o) continue;
            double vx = pos[3 * s] - pos[3 * o], vy = pos[3 * s + 1] - pos[3 * o + 1];
            double vz = pos[3 * s + 2] - pos[3 * o + 2];
            if (vx == 0.0 && vy == 0.0 && vz == 0.0) continue;
            h[L - 1][fx_vec2pix(nsm, vx, vy, vz)] += 1;
        }
        for (int32_t k = L - 1; k > 0; --k)
            for (int64_t p = 0; p < npix[k]; ++p) h[k - 1][par[k][p]] += h[k][p];
        or_leaf* leaves = (or_leaf*)malloc(sizeof(or_leaf) * (size_t)R);
        int64_t nl = 0;
        int64_t nact = npix[0] / 2;
        or_key* act = (or_key*)malloc(sizeof(or_key) * (size_t)(npix[L - 1]));
        int64_t a = 0;
        for (int64_t p = 0; p < npix[0]; ++p)
            if (anti[0][p] > p) { act[a].pix = p; act[a].cnt = h[0][p] + h[0][anti[0][p]]; ++a; }
        for (int32_t k = 0; k < L; ++k) {
            if (k == L - 1) {
                for (int64_t i = 0; i < nact; ++i) { leaves[nl].level = lmin + k; leaves[nl].pix = act[i].pix; ++nl; }
                break;
            }
            qsort(act, (size_t)nact, sizeof(or_key), key_cmp);
            int64_t nref = nact / 2;
            for (int64_t i = nref; i < nact; ++i) { leaves[nl].level = lmin + k; leaves[nl].pix = act[i].pix; ++nl; }
            /* children of the refined pairs: the level-(k+1) pixels whose parent is the canonical pixel */
            or_key* nxt = (or_key*)malloc(sizeof(or_key) * (size_t)(4 * nref));
            int64_t b = 0;
            for (int64_t c = 0; c < npix[k + 1]; ++c) {
                int64_t pc = par[k + 1][c];
                for (int64_t i = 0; i < nref; ++i)
                    if (act[i].pix == pc) {
                        int64_t cc = c < anti[k + 1][c] ? c : anti[k + 1][c];
                        nxt[b].pix = cc;
                        nxt[b].cnt = h[k + 1][cc] + h[k + 1][anti[k + 1][cc]];
                        ++b;
                        break;
                    }
            }
            memcpy(act, nxt, sizeof(or_key) * (size_t)b);
            free(nxt);
            nact = b;
        }
        qsort(leaves, (size_t)nl, sizeof(or_leaf), leaf_cmp);
        for (int64_t r = 0; r < nl && r < R; ++r) {
            int64_t ns = 1LL << leaves[r].level;
            if (pix_out) pix_out[oi * R + r] = leaves[r].pix;
            if (level_out) level_out[oi * R + r] = leaves[r].level;
            if (dirs_out) or_hp_pix2vec(ns, leaves[r].pix, dirs_out + 3 * (oi * R + r));
            if (w2_out) w2_out[oi * R + r] = 2.0 / (double)(12 * ns * ns);
        }
        free(leaves);
        free(act);
        for (int32_t k = 0; k < L; ++k) free(h[k]);
        free(h);
    }
    for (int32_t k = 0; k < L; ++k) { free(anti[k]); free(par[k]); }
    free(anti); free(par); free(npix);
    return R;
}

/* ---------------------------------------------------------------- tracing */

/* Trace one ray from `origin` along unit direction d (Section 2.1, Fig. 2).
 * From the current point c with projection Zc, every neighbour k with
 *     Z_k = R.d,  R = x_k - x_origin,
 * strictly greater than Zc is a forward candidate; its squared distance to
 * the ray axis is D_k = |q|^2 with q = R - Z_k d.  Both are evaluated in FP64
 * with explicit fused multiply-adds, x first:
 *     Z_k = fma(R.z, d.z, fma(R.y, d.y, R.x d.x)),  q.i = fma(-Z_k, d.i, R.i),
 *     D_k = fma(q.z, q.z, fma(q.y, q.y, q.x q.x)).  The ray
 * steps to the candidate of least D_k (equal D: smaller point id), records
 * (k, Z_k), and continues from k with Zc = Z_k.  It ends where no neighbour
 * is forward.  The origin is not recorded.  Returns the number of points;
 * writes at most `cap` of them. */
OR_API int64_t or_trace_ray(const double* pos, const int64_t* off, const int32_t* idx, int64_t P,
                            int64_t origin, const double* d, int32_t* ids, double* Z, int64_t cap) {
    const double ox = pos[3 * origin], oy = pos[3 * origin + 1], oz = pos[3 * origin + 2];
    int64_t c = origin, n = 0;
    double Zc = 0.0;
    for (int64_t step = 0; step < P; ++step) {
        int64_t best = -1;
        double bestD = 0.0, bestZ = 0.0;
        for (int64_t e = off[c]; e < off[c + 1]; ++e) {
            int64_t k = idx[e];
            double Rx = pos[3 * k] - ox, Ry = pos[3 * k + 1] - oy, Rz = pos[3 * k + 2] - oz;
            double Zk = fma(Rz, d[2], fma(Ry, d[1], Rx * d[0]));
            if (!(Zk > Zc)) continue;
            double qx = fma(-Zk, d[0], Rx), qy = fma(-Zk, d[1], Ry), qz = fma(-Zk, d[2], Rz);
            double Dk = fma(qz, qz, fma(qy, qy, qx * qx));
            if (best < 0 || Dk < bestD || (Dk == bestD && k < best)) {
                best = k; bestD = Dk; bestZ = Zk;
            }
        }
        if (best < 0) break;
        if (n < cap) { ids[n] = (int32_t)best; Z[n] = bestZ; }
        ++n;
        c = best;
        Zc = bestZ;
    }
    return n;
}

/* Trace every ray of every listed origin.  Ray slot s = o*2R + 2r (+n_r) or
 * 2r+1 (-n_r), o the position in `origins`.  ray_off[s+1]-ray_off[s] is the
 * ray's length; lists are concatenated in slot order.  If ids/Z are NULL only
 * ray_off is written.  Returns the total number of entries. */
OR_API int64_t or_trace_all(const double* pos, const int64_t* off, const int32_t* idx, int64_t P,
                            int64_t R, const double* dirs, int32_t per_origin_dirs,
                            const int32_t* origins, int64_t n_origins,
                            int64_t* ray_off, int32_t* ids, double* Z, int nthreads) {
    const int64_t nr = n_origins * 2 * R;
    int64_t* len = (int64_t*)calloc((size_t)nr, sizeof(int64_t));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t o = 0; o < n_origins; ++o) {
        const double* dv = per_origin_dirs ? dirs + 3 * R * o : dirs;
        for (int64_t r = 0; r < R; ++r) {
            double dp[3] = {dv[3 * r], dv[3 * r + 1], dv[3 * r + 2]};
            double dm[3] = {-dp[0], -dp[1], -dp[2]};
            len[o * 2 * R + 2 * r] = or_trace_ray(pos, off, idx, P, origins[o], dp, NULL, NULL, 0);
            len[o * 2 * R + 2 * r + 1] = or_trace_ray(pos, off, idx, P, origins[o], dm, NULL, NULL, 0);
        }
    }
    ray_off[0] = 0;
    for (int64_t s = 0; s < nr; ++s) ray_off[s + 1] = ray_off[s] + len[s];
    free(len);
    if (ids && Z) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
        for (int64_t o = 0; o < n_origins; ++o) {
            const double* dv = per_origin_dirs ? dirs + 3 * R * o : dirs;
            for (int64_t r = 0; r < R; ++r) {
                double dp[3] = {dv[3 * r], dv[3 * r + 1], dv[3 * r + 2]};
                double dm[3] = {-dp[0], -dp[1], -dp[2]};
                int64_t sp = o * 2 * R + 2 * r, sm = sp + 1;
                or_trace_ray(pos, off, idx, P, origins[o], dp, ids + ray_off[sp], Z + ray_off[sp],
                             ray_off[sp + 1] - ray_off[sp]);
                or_trace_ray(pos, off, idx, P, origins[o], dm, ids + ray_off[sm], Z + ray_off[sm],
                             ray_off[sm + 1] - ray_off[sm]);
            }
        }
    }
    return ray_off[nr];
}

/* --------------------------------------------------------- Feautrier solve */

/* u at row m of the discrete second-order Feautrier system (eq. 1) on a line
 * of N points with optical-depth increments dtau[0..N-2] and source S[0..N-1].
 *
 * Interior rows 0<d<N-1 (three-point second difference on a non-uniform grid):
 *   -A_d u_{d-1} + (1 + A_d + C_d) u_d - C_d u_{d+1} = S_d,
 *   A_d = 2/(dtau_{d-1}(dtau_{d-1}+dtau_d)),  C_d = 2/(dtau_d(dtau_{d-1}+dtau_d)).
 * Boundary rows (second order, incoming intensity I at both ends):
 *   (1 + 2/dt + 2/dt^2) u_0 - (2/dt^2) u_1 = S_0 + 2 I/dt,  dt = dtau_0, and the mirror
 *   image at d = N-1 with dt = dtau_{N-2}.
 * The system is eliminated from both ends towards m in the rescaled form
 * u_{d} = u_{d+1}/(1+F_d) + Z_d (forward) and u_d = u_{d-1}/(1+G_d) + W_d
 * (backward), where every F, G, Z, W is a sum and quotient of positive terms,
 * so no cancellation occurs for small dtau.  N == 1 returns I. */
OR_API double or_feautrier_u(int64_t N, int64_t m, const double* dtau, const double* S, double I) {
    if (N == 1) return I;
    double F = 0.0, Zf = 0.0, G = 0.0, W = 0.0;
    /* forward sweep over rows 0 .. m-1 */
    for (int64_t d = 0; d < m; ++d) {
        if (d == 0) {
            double dt = dtau[0];
            double C0 = 2.0 / (dt * dt);
            F = dt * (1.0 + 0.5 * dt);
            Zf = (S[0] + 2.0 * I / dt) / (C0 * (1.0 + F));
        } else {
            double a = dtau[d - 1], b = dtau[d];
            double A = 2.0 / (a * (a + b)), C = 2.0 / (b * (a + b));
            double Fn = (1.0 + A * F / (1.0 + F)) / C;
            Zf = (S[d] + A * Zf) / (C * (1.0 + Fn));
            F = Fn;
        }
    }
    /* backward sweep over rows N-1 .. m+1 */
    for (int64_t d = N - 1; d > m; --d) {
        if (d == N - 1) {
            double dt = dtau[N - 2];
            double AN = 2.0 / (dt * dt);
            G = dt * (1.0 + 0.5 * dt);
            W = (S[N - 1] + 2.0 * I / dt) / (AN * (1.0 + G));
        } else {
            double a = dtau[d - 1], b = dtau[d];
            double A = 2.0 / (a * (a + b)), C = 2.0 / (b * (a + b));
            double Gn = (1.0 + C * G / (1.0 + G)) / A;
            W = (S[d] + C * W) / (A * (1.0 + Gn));
            G = Gn;
        }
    }
    if (m == 0) {
        double dt = dtau[0];
        double C0 = 2.0 / (dt * dt);
        return (S[0] + 2.0 * I / dt + C0 * W) / (1.0 + 2.0 / dt + C0 * G / (1.0 + G));
    }
    if (m == N - 1) {
        double dt = dtau[N - 2];
        double AN = 2.0 / (dt * dt);
        return (S[N - 1] + 2.0 * I / dt + AN * Zf) / (1.0 + 2.0 / dt + AN * F / (1.0 + F));
    }
    double a = dtau[m - 1], b = dtau[m];
    double A = 2.0 / (a * (a + b)), C = 2.0 / (b * (a + b));
    return (S[m] + A * Zf + C * W) / (1.0 + A * F / (1.0 + F) + C * G / (1.0 + G));
}

/* u at row m of the fourth-order Hermitian discretisation of the same equation
 * (the scheme of Auer 1976 that the paper names for its solver, Section 2.1;
 * the paper gives no formulas, so the rows are derived here).
 *
 * Interior rows: with f = u - S = u" (eq. 1) and the outer and inner steps
 * a = dtau_{d-1}, b = dtau_d, the compact relation
 *   (u_{d+1} - u_d)/b - (u_d - u_{d-1})/a = w_- f_{d-1} + w_0 f_d + w_+ f_{d+1}
 * is exact for every polynomial u of degree <= 4 when
 *   w_- = (a^3 + 2a^2 b - b^3) / (12 a (a+b)),  w_+ = (b^3 + 2a b^2 - a^3) / (12 b (a+b)),
 *   w_- + w_0 + w_+ = (a+b)/2
 * (h/12, 10h/12, h/12 on a uniform grid).  Divided by (a+b)/2, with
 * alpha, beta, gamma = w_-, w_0, w_+ over (a+b)/2 and A, C the second-order
 * coefficients above:
 *   -(A - alpha) u_{d-1} + (1 + A - alpha + C - gamma) u_d - (C - gamma) u_{d+1}
 *      = alpha S_{d-1} + beta S_d + gamma S_{d+1}.
 * Boundary rows (third order): the second-order condition with the next
 * Taylor term, u''' = u' - S', the slope of S taken one-sided:
 *   (u_1 - u_0)/dt = (u_0 - I)(1 + dt^2/6) + (dt/2)(u_0 - S_0) - (dt/6)(S_1 - S_0),
 * i.e. (1 + E + 2/dt^2) u_0 - (2/dt^2) u_1 = S_0 + E I + (S_1 - S_0)/3 with
 * E = (2/dt)(1 + dt^2/6); the mirror image at d = N-1.
 * The system is eliminated from both ends towards m in the same rescaled form
 * as the second-order rows (u_d = u_{d+1}/(1+F_d) + Z_d forward, the mirror image
 * backward), which loses nothing to cancellation for small steps as long as
 * the off-diagonals -(A - alpha), -(C - gamma) are non-positive: true while every
 * step is below about 3.46 (2 sqrt 3 on a uniform grid); a row beyond that limit
 * makes the result NaN (the caller keeps steps small, e.g. with dtau_max).
 * The weights assume S smooth in tau: between very unequal steps the weight of
 * the far neighbour grows like -(long step)/(6 short step) and amplifies jumps
 * of S.  Since alpha + beta + gamma = 1 the right-hand side is evaluated as
 * S_d + alpha (S_{d-1} - S_d) + gamma (S_{d+1} - S_d), the same value without
 * the large, nearly cancelling products beta S_d and gamma S_{d+1} that unequal
 * steps would bring into its rounding.  N == 1 returns I. */
OR_API double or_feautrier_u_hermite(int64_t N, int64_t m, const double* dtau, const double* S, double I) {
    if (N == 1) return I;
    /* row d: -Am u_{d-1} + (1 + Am + Cp) u_d - Cp u_{d+1} = Rd; the end rows have
     * (Am, Cp) = (0, K) at d = 0 and (K, 0) at d = N-1 and an extra E on the diagonal */
#define OR_HERM_ROW(d, Am, Cp, Ex, Rd)                                                         \
    do {                                                                                       \
        if ((d) == 0 || (d) == N - 1) {                                                        \
            const double dt_ = (d) == 0 ? dtau[0] : dtau[N - 2];                               \
            const int64_t nb_ = (d) == 0 ? 1 : N - 2;                                          \
            const double K_ = 2.0 / (dt_ * dt_);                                               \
            Ex = (2.0 / dt_) * (1.0 + dt_ * dt_ / 6.0);                                        \
            Am = (d) == 0 ? 0.0 : K_;                                                          \
            Cp = (d) == 0 ? K_ : 0.0;                                                          \
            Rd = S[d] + Ex * I + (S[nb_] - S[d]) / 3.0;                                        \
        } else {                                                                               \
            const double a_ = dtau[(d) - 1], b_ = dtau[d], h_ = 0.5 * (a_ + b_);               \
            const double wm_ = (a_ * a_ * a_ + 2.0 * a_ * a_ * b_ - b_ * b_ * b_) / (12.0 * a_ * (a_ + b_)); \
            const double wp_ = (b_ * b_ * b_ + 2.0 * a_ * b_ * b_ - a_ * a_ * a_) / (12.0 * b_ * (a_ + b_)); \
            const double al_ = wm_ / h_, ga_ = wp_ / h_;                                       \
            Am = 2.0 / (a_ * (a_ + b_)) - al_;                                                 \
            Cp = 2.0 / (b_ * (a_ + b_)) - ga_;                                                 \
            Ex = 0.0;                                                                          \
            Rd = S[d] + al_ * (S[(d) - 1] - S[d]) + ga_ * (S[(d) + 1] - S[d]);                 \
            if (!(Am >= 0.0) || !(Cp > 0.0)) bad = 1;                                          \
        }                                                                                      \
    } while (0)
    int bad = 0;
    /* forward over rows 0 .. m-1: u_d = u_{d+1}/(1+F) + Z */
    double F = 0.0, Z = 0.0;
    for (int64_t d = 0; d < m; ++d) {
        double Am, Cp, Ex, Rd;
        OR_HERM_ROW(d, Am, Cp, Ex, Rd);
        const double Fn = (1.0 + Ex + Am * F / (1.0 + F)) / Cp;
        Z = (Rd + Am * Z) / (Cp * (1.0 + Fn));
        F = Fn;
    }
    /* backward over rows N-1 .. m+1: u_d = u_{d-1}/(1+G) + W */
    double G = 0.0, W = 0.0;
    for (int64_t d = N - 1; d > m; --d) {
        double Am, Cp, Ex, Rd;
        OR_HERM_ROW(d, Am, Cp, Ex, Rd);
        const double Gn = (1.0 + Ex + Cp * G / (1.0 + G)) / Am;
        W = (Rd + Cp * W) / (Am * (1.0 + Gn));
        G = Gn;
    }
    double Am, Cp, Ex, Rd;
    OR_HERM_ROW(m, Am, Cp, Ex, Rd);
#undef OR_HERM_ROW
    if (bad) return NAN;  /* a step beyond the rows' limit: no value (the caller reports it) */
    /* row m with u_{m-1} = u_m/(1+F) + Z and u_{m+1} = u_m/(1+G) + W */
    return (Rd + Am * Z + Cp * W) / (1.0 + Ex + Am * F / (1.0 + F) + Cp * G / (1.0 + G));
}

/* ------------------------------------------------------- full J at origins */

typedef struct {
    int64_t cap;
    int32_t* idm; double* Zm;   /* backward ray (-n) */
    int32_t* idp; double* Zp;   /* forward ray  (+n) */
    int32_t* q;   double* s;    /* assembled line */
    double* dtau; double* S; double* chi; double* eta;
    int64_t* k; double* t;
    int64_t* nsub;              /* optical-depth sub-steps per interval */
    int64_t rcap;               /* line refined by optical-depth sub-steps */
    double* rdtau; double* rS; double* rchi;
    int64_t vcap;               /* line after velocity sampling: point i lies between */
    int32_t* va; int32_t* vb;   /* assembled points va[i] and vb[i] at weight vw[i] */
    double* vw; double* vdot;   /* (0 for an assembled point), projected velocity, */
    double* vds;                /* length of the interval to point i+1 */
    int64_t* vk; double* vt;    /* shift of point i in the current block */
    double* vchi; double* veta; double* vS;
    int64_t* vn;                /* velocity sub-steps per assembled interval */
} or_ws;

static void ws_grow(or_ws* w, int64_t n) {
    if (n <= w->cap) return;
    int64_t c = n * 2;
    w->idm = realloc(w->idm, c * sizeof(int32_t)); w->Zm = realloc(w->Zm, c * sizeof(double));
    w->idp = realloc(w->idp, c * sizeof(int32_t)); w->Zp = realloc(w->Zp, c * sizeof(double));
    w->q = realloc(w->q, (2 * c + 1) * sizeof(int32_t)); w->s = realloc(w->s, (2 * c + 1) * sizeof(double));
    w->dtau = realloc(w->dtau, (2 * c + 1) * sizeof(double)); w->S = realloc(w->S, (2 * c + 1) * sizeof(double));
    w->chi = realloc(w->chi, (2 * c + 1) * sizeof(double)); w->eta = realloc(w->eta, (2 * c + 1) * sizeof(double));
    w->k = realloc(w->k, (2 * c + 1) * sizeof(int64_t)); w->t = realloc(w->t, (2 * c + 1) * sizeof(double));
    w->vn = realloc(w->vn, (2 * c + 1) * sizeof(int64_t));
    w->cap = c;
}

static void ws_free(or_ws* w) {
    free(w->idm); free(w->Zm); free(w->idp); free(w->Zp); free(w->q); free(w->s);
    free(w->dtau); free(w->S); free(w->chi); free(w->eta); free(w->k); free(w->t);
    free(w->rdtau); free(w->rS); free(w->rchi);
    free(w->va); free(w->vb); free(w->vw); free(w->vdot); free(w->vds);
    free(w->vk); free(w->vt); free(w->vchi); free(w->veta); free(w->vS); free(w->vn); free(w->nsub);
}

static void ws_grow_vel(or_ws* w, int64_t n) {
    if (n <= w->vcap) return;
    int64_t c = n * 2;
    w->va = realloc(w->va, c * sizeof(int32_t)); w->vb = realloc(w->vb, c * sizeof(int32_t));
    w->vw = realloc(w->vw, c * sizeof(double)); w->vdot = realloc(w->vdot, c * sizeof(double));
    w->vds = realloc(w->vds, c * sizeof(double));
    w->vk = realloc(w->vk, c * sizeof(int64_t)); w->vt = realloc(w->vt, c * sizeof(double));
    w->vchi = realloc(w->vchi, c * sizeof(double)); w->veta = realloc(w->veta, c * sizeof(double));
    w->vS = realloc(w->vS, c * sizeof(double)); w->nsub = realloc(w->nsub, c * sizeof(int64_t));
    w->vcap = c;
}

static void ws_grow_refined(or_ws* w, int64_t n) {
    if (n <= w->rcap) return;
    int64_t c = n * 2;
    w->rdtau = realloc(w->rdtau, c * sizeof(double));
    w->rS = realloc(w->rS, c * sizeof(double));
    w->rchi = realloc(w->rchi, c * sizeof(double));
    w->rcap = c;
}

/* Adaptive optical-depth increments (Section 2.1.2, eq. 2).  The interval
 * between line points d and d+1 is split into
 *     n_d = ceil(max(chi_d, chi_{d+1}) ds_d / dtau_max)
 * equal parts (computed as (max * ds) * (1/dtau_max), the reciprocal rounded
 * once; n_d clamped to 1 .. max_sub; ds_d the interval's length), and chi and eta are interpolated
 * linearly on the sub-intervals: at w = i/n_d, chi = (1-w) chi_d + w chi_{d+1},
 * eta likewise, S = eta/chi.  Every sub-interval gets the trapezoid
 * dtau = (0.5 (chi_j + chi_{j+1})) (ds_d / n_d).  Writes the refined line into
 * w->rdtau / w->rS and returns its length; *m_out receives the refined index of
 * line point m.  dtau_max <= 0 leaves every interval whole. */
static int64_t refine_line(or_ws* w, int64_t N, int64_t m, double dtau_max, int64_t max_sub, int64_t* m_out) {
    const double rdt = dtau_max > 0.0 ? 1.0 / dtau_max : 0.0;
    int64_t total = 1;
    for (int64_t d = 0; d + 1 < N; ++d) {
        int64_t n = 1;
        if (dtau_max > 0.0) {
            const double ds = w->vds[d];
            const double cm = w->vchi[d] > w->vchi[d + 1] ? w->vchi[d] : w->vchi[d + 1];
            double c = ceil((cm * ds) * rdt);
            if (c > (double)max_sub) c = (double)max_sub;
            n = c >= 1.0 ? (int64_t)c : 1;
        }
        w->nsub[d] = n;
        total += n;
    }
    ws_grow_refined(w, total);
    int64_t j = 0;
    for (int64_t d = 0; d < N; ++d) {
        if (d == m) *m_out = j;
        w->rS[j] = w->vS[d];
        w->rchi[j] = w->vchi[d];
        ++j;
        if (d + 1 == N) break;
        const int64_t n = w->nsub[d];
        for (int64_t i = 1; i < n; ++i) {
            const double wt = (double)i / (double)n;
            const double c = (1.0 - wt) * w->vchi[d] + wt * w->vchi[d + 1];
            const double e = (1.0 - wt) * w->veta[d] + wt * w->veta[d + 1];
            w->rS[j] = e / c;
            w->rchi[j] = c;
            ++j;
        }
    }
    j = 0;
    for (int64_t d = 0; d + 1 < N; ++d) {
        const int64_t n = w->nsub[d];
        const double h = w->vds[d] / (double)n;
        for (int64_t i = 0; i < n; ++i, ++j) w->rdtau[j] = (0.5 * (w->rchi[j] + w->rchi[j + 1])) * h;
    }
    return total;
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Adaptive velocity sampling (Section 2.1.1).  With p_d = n_r . (v_{q_d} - v_o)
 * the projected velocity of assembled line point d (in Doppler widths), the
 * interval d .. d+1 is split into
 *     m_d = ceil(|p_{d+1} - p_d| / dv_max)
 * equal parts (the product with the reciprocal of dv_max rounded once; m_d
 * clamped to 1 .. max_sub).  A point at weight w = j/m_d carries the projected
 * velocity (1-w) p_d + w p_{d+1}; its optics are (1-w) X_d + w X_{d+1}, where
 * X_e is point e's table interpolated at that point's own shift (so the line
 * profile moves smoothly along the interval), and each part is ds_d / m_d long.
 * Fills w->va/vb/vw/vdot/vds for the sampled line, returns its length and the
 * new index of the origin in *m_out.  dv_max <= 0 (or a static medium) keeps
 * the assembled points. */
static int64_t velocity_line(or_ws* w, int64_t N, int64_t m, const float* vel, int64_t o, const double* dp,
                             double dv_max, int64_t max_sub, int64_t* m_out) {
    /* projected velocities of the assembled points, kept in w->t (re-filled per block later) */
    for (int64_t d = 0; d < N; ++d) {
        if (vel) {
            const float* vq = vel + 3 * (int64_t)w->q[d];
            const float* vo = vel + 3 * o;
            double dvx = (double)vq[0] - (double)vo[0];
            double dvy = (double)vq[1] - (double)vo[1];
            double dvz = (double)vq[2] - (double)vo[2];
            w->t[d] = (dp[0] * dvx + dp[1] * dvy) + dp[2] * dvz;
        } else {
            w->t[d] = 0.0;
        }
    }
    const double rdv = dv_max > 0.0 ? 1.0 / dv_max : 0.0;
    int64_t total = 1;
    for (int64_t d = 0; d + 1 < N; ++d) {
        int64_t n = 1;
        if (dv_max > 0.0 && vel) {
            double c = ceil(fabs(w->t[d + 1] - w->t[d]) * rdv);
            if (c > (double)max_sub) c = (double)max_sub;
            n = c >= 1.0 ? (int64_t)c : 1;
        }
        w->vn[d] = n;
        total += n;
    }
    ws_grow_vel(w, total);
    int64_t i = 0;
    for (int64_t d = 0; d < N; ++d) {
        if (d == m) *m_out = i;
        w->va[i] = (int32_t)d;
        w->vb[i] = (int32_t)d;
        w->vw[i] = 0.0;
        w->vdot[i] = w->t[d];
        ++i;
        if (d + 1 == N) break;
        const int64_t n = w->vn[d];
        const double h = (w->s[d + 1] - w->s[d]) / (double)n;
        w->vds[i - 1] = h;
        for (int64_t j = 1; j < n; ++j) {
            const double wt = (double)j / (double)n;
            w->va[i] = (int32_t)d;
            w->vb[i] = (int32_t)(d + 1);
            w->vw[i] = wt;
            w->vdot[i] = (1.0 - wt) * w->t[d] + wt * w->t[d + 1];
            w->vds[i] = h;
            ++i;
        }
    }
    return total;
}

/* J[o][f] at every listed origin (eq. 3, eq. 4).
 *
 * For each antipodal pair r (direction n_r and its negation) the two rays
 * are traced, the line is assembled as reverse(backward list), origin,
 * forward list, with coordinate s = (-Z_back reversed, 0, Z_fwd) and
 * ds_d = s_{d+1} - s_d.  Optics in the comoving frame of the origin along
 * +n_r (Section 2.1.1): the shift of line point q in block b is
 *     delta_q = (n_r . (v_q - v_o)) / dx_b,  k = floor(delta_q), t = delta_q - k,
 *     chi'_q[f] = (1-t) chi_q[clamp(f-k)] + t chi_q[clamp(f-k-1)]
 * with indices clamped to the block; eta the same; S = eta'/chi'.  The
 * optical-depth increment is the trapezoid dtau_d = (0.5 (chi'_d + chi'_{d+1})) ds_d.
 * u at the origin comes from or_feautrier_u; J accumulates w2[r] u in ascending r.
 *
 * dirs: [R][3] shared, or [n_origins][R][3] when per_origin_dirs; w2 likewise.
 * vel may be NULL (static).  u_out, if not NULL, receives u[o][r][f]. */
OR_API int or_compute_J_sub(int64_t P, const double* pos, const int64_t* off, const int32_t* idx,
                            const float* vel, int64_t F, int32_t nblk, const int32_t* blk_len,
                            const double* blk_dx, const double* chi, const double* eta, int64_t ld,
                            const double* I_bc, int64_t R, const double* dirs, const double* w2,
                            int32_t per_origin_dirs, const int32_t* origins, int64_t n_origins,
                            double dv_max, double dtau_max, int64_t max_sub, int32_t scheme, double* J,
                            double* u_out, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int err = 0;
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        or_ws w;
        memset(&w, 0, sizeof(w));
        ws_grow(&w, 256);
        ws_grow_vel(&w, 512);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t oi = 0; oi < n_origins; ++oi) {
            const int64_t o = origins[oi];
            const double* dv = per_origin_dirs ? dirs + 3 * R * oi : dirs;
            const double* wv = per_origin_dirs ? w2 + R * oi : w2;
            double* Jo = J + oi * F;
            for (int64_t f = 0; f < F; ++f) Jo[f] = 0.0;
            for (int64_t r = 0; r < R; ++r) {
                double dp[3] = {dv[3 * r], dv[3 * r + 1], dv[3 * r + 2]};
                double dm[3] = {-dp[0], -dp[1], -dp[2]};
                int64_t np_, nm;
                for (;;) {
                    np_ = or_trace_ray(pos, off, idx, P, o, dp, w.idp, w.Zp, w.cap);
                    nm = or_trace_ray(pos, off, idx, P, o, dm, w.idm, w.Zm, w.cap);
                    if (np_ <= w.cap && nm <= w.cap) break;
                    ws_grow(&w, (np_ > nm ? np_ : nm));
                }
                /* line assembly */
                const int64_t N = nm + 1 + np_, m = nm;
                for (int64_t j = 0; j < nm; ++j) {
                    w.q[j] = w.idm[nm - 1 - j];
                    w.s[j] = -w.Zm[nm - 1 - j];
                }
                w.q[m] = (int32_t)o;
                w.s[m] = 0.0;
                for (int64_t j = 0; j < np_; ++j) {
                    w.q[m + 1 + j] = w.idp[j];
                    w.s[m + 1 + j] = w.Zp[j];
                }
                int64_t mv = m;
                const int64_t Nv = velocity_line(&w, N, m, vel, o, dp, dv_max, max_sub, &mv);
                int64_t fb = 0;
                for (int32_t b = 0; b < nblk; ++b) {
                    const int64_t L = blk_len[b];
                    /* per-point Doppler shift in this block's index units */
                    for (int64_t i = 0; i < Nv; ++i) {
                        if (vel) {
                            double delta = w.vdot[i] / blk_dx[b];
                            double fl = floor(delta);
                            w.vk[i] = (int64_t)fl;
                            w.vt[i] = delta - fl;
                        } else {
                            w.vk[i] = 0;
                            w.vt[i] = 0.0;
                        }
                    }
                    for (int64_t j = 0; j < L; ++j) {
                        const int64_t f = fb + j;
                        for (int64_t i = 0; i < Nv; ++i) {
                            const double* ca = chi + (int64_t)w.q[w.va[i]] * ld + fb;
                            const double* ea = eta + (int64_t)w.q[w.va[i]] * ld + fb;
                            const double* cb = chi + (int64_t)w.q[w.vb[i]] * ld + fb;
                            const double* eb = eta + (int64_t)w.q[w.vb[i]] * ld + fb;
                            int64_t ia = clampi(j - w.vk[i], 0, L - 1);
                            int64_t ib = clampi(j - w.vk[i] - 1, 0, L - 1);
                            double t = w.vt[i], wt = w.vw[i];
                            /* each end point's table at this point's shift, then mixed by weight */
                            const double xa = (1.0 - t) * ca[ia] + t * ca[ib];
                            const double xb = (1.0 - t) * cb[ia] + t * cb[ib];
                            const double ya = (1.0 - t) * ea[ia] + t * ea[ib];
                            const double yb = (1.0 - t) * eb[ia] + t * eb[ib];
                            w.vchi[i] = (1.0 - wt) * xa + wt * xb;
                            w.veta[i] = (1.0 - wt) * ya + wt * yb;
                            w.vS[i] = w.veta[i] / w.vchi[i];
                        }
                        double u;
                        if (dtau_max > 0.0) {
                            int64_t mr = 0;
                            const int64_t Nr = refine_line(&w, Nv, mv, dtau_max, max_sub, &mr);
                            u = scheme == 1 ? or_feautrier_u_hermite(Nr, mr, w.rdtau, w.rS, I_bc[f])
                                            : or_feautrier_u(Nr, mr, w.rdtau, w.rS, I_bc[f]);
                        } else {
                            ws_grow_refined(&w, Nv);
                            for (int64_t i = 0; i + 1 < Nv; ++i)
                                w.rdtau[i] = (0.5 * (w.vchi[i] + w.vchi[i + 1])) * w.vds[i];
                            u = scheme == 1 ? or_feautrier_u_hermite(Nv, mv, w.rdtau, w.vS, I_bc[f])
                                            : or_feautrier_u(Nv, mv, w.rdtau, w.vS, I_bc[f]);
                        }
                        if (!(u == u)) err = 1;
                        if (u_out) u_out[(oi * R + r) * F + f] = u;
                        Jo[f] += wv[r] * u;
                    }
                    fb += L;
                }
            }
        }
        ws_free(&w);
    }
    return err ? -7 : 0;
}

/* J without optical-depth sub-steps (every interval whole). */
OR_API int or_compute_J(int64_t P, const double* pos, const int64_t* off, const int32_t* idx,
                        const float* vel, int64_t F, int32_t nblk, const int32_t* blk_len,
                        const double* blk_dx, const double* chi, const double* eta, int64_t ld,
                        const double* I_bc, int64_t R, const double* dirs, const double* w2,
                        int32_t per_origin_dirs, const int32_t* origins, int64_t n_origins,
                        double* J, double* u_out, int nthreads) {
    return or_compute_J_sub(P, pos, off, idx, vel, F, nblk, blk_len, blk_dx, chi, eta, ld, I_bc, R, dirs, w2,
                            per_origin_dirs, origins, n_origins, 0.0, 0.0, 1, 0, J, u_out, nthreads);
}
