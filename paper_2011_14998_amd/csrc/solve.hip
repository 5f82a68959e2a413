// Feautrier sweep and J reduction.
//
// Work item = (origin, antipodal pair, 64-frequency chunk); one wavefront per
// item, one frequency per lane.  The line of a pair is
//     reverse(ray -n_r), origin, ray +n_r
// and only u at the origin is needed, so each side is eliminated from its far
// end inwards (second-order Feautrier equation, eq. 1, with second-order
// boundary conditions at both ends) and the two sides meet at the origin.
// The fourth-order (Hermitian) rows are an option with the same structure
// (below, at row_h).
// Nothing but the running (F, Z) pair and the previous point's optics is kept
// per lane: a line of any length streams through registers.
//
// Rescaled elimination.  With the three-point rows
//     -A_d u_{d-1} + (1 + A_d + C_d) u_d - C_d u_{d+1} = S_d,
//     A_d = 2/(a(a+b)), C_d = 2/(b(a+b)),  a = outer dtau, b = inner dtau,
// and u_d = u_{d+1}/(1+F_d) + Z_d, the recurrences are
//     F_d = b(a+b)/2 + (b/a) F_{d-1}/(1+F_{d-1})
//     Z_d = (b(a+b)/2 S_d + (b/a) Z_{d-1}) / (1 + F_d)
// and at the far end (boundary row from u' = u - I to second order)
//     F_0 = b(1 + b/2),  Z_0 = (b^2/2 S_0 + b I)/(1 + F_0).
// Carried per unit inner step, F_d = b G_d and Z_d = b Y_d, and since the
// outer step a of row d is the inner step of row d-1, the ratio b/a cancels:
//     G_d = (a+b)/2 + G_{d-1} r_{d-1},   r_d = 1/(1 + b G_d),
//     Y_d = ((a+b)/2 S_d + Y_{d-1}) r_d,
//     G_0 = 1 + b/2,  Y_0 = (b/2 S_0 + I) r_0.
// One reciprocal per row, and the only coefficient, (a+b)/2, is the correctly
// rounded exact value in any precision (an FP32 evaluation equals the FP64
// one rounded once), however small the steps.  Every term is a sum or product
// of positive numbers, so small optical-depth steps lose nothing to
// cancellation.  At the origin (a, b the steps to the two sides' last rows)
//     u = ((a+b)/2 S + Y_- + Y_+) / ((a+b)/2 + G_- r_- + G_+ r_+),
// and with one side empty (dtau t on the other)
//     u = (t/2 S + I + Y) / (1 + t/2 + G r).
//
// Per-point data that is the same for every frequency (point id, ds, the
// velocity projection) is loaded for 64 points at once, one per lane, and
// broadcast with readlane; each lane then gathers its own chi/eta values of
// that point's row -- 64 consecutive values, one coalesced 256-byte read per
// table for FP32.
#include "rt_internal.h"

#include <type_traits>

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

__device__ inline int64_t readlane_64(int64_t v, int j) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_readlane(p.x, j);
    p.y = __builtin_amdgcn_readlane(p.y, j);
    return __builtin_bit_cast(int64_t, p);
}

// Values every lane holds identically, moved to scalar registers so that the
// compiler keeps loop bounds and branches on them scalar.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uni64(int64_t v) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_readfirstlane(p.x);
    p.y = __builtin_amdgcn_readfirstlane(p.y);
    return __builtin_bit_cast(int64_t, p);
}

template <typename T>
__device__ inline T readlane_t(T v, int j);
template <>
__device__ inline float readlane_t<float>(float v, int j) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j));
}
template <>
__device__ inline double readlane_t<double>(double v, int j) { return readlane_d(v, j); }

struct LaneFreq {
    int f;       // global frequency index of this lane (clamped to F-1 when inactive)
    bool active;
    int fb;      // start of the lane's block
    int L;       // length of the block
    int fl;      // index inside the block
    double inv_dx;
    double dx;
};

__device__ inline LaneFreq lane_freq_at(const SolveLaunch& a, int f) {
    LaneFreq lf;
    lf.active = f < a.F;
    lf.f = lf.active ? f : a.F - 1;
    int b = 0;
#pragma unroll
    for (int bb = 1; bb < RT_MAX_FREQ_BLOCKS; ++bb)
        if (bb < a.n_blocks && lf.f >= a.blk_start[bb]) b = bb;
    int fb = a.blk_start[0], nb = a.blk_start[1];
    double idx = a.inv_dx[0], dxb = a.dx[0];
#pragma unroll
    for (int bb = 1; bb < RT_MAX_FREQ_BLOCKS; ++bb)
        if (bb == b) {
            fb = a.blk_start[bb];
            nb = a.blk_start[bb + 1];
            idx = a.inv_dx[bb];
            dxb = a.dx[bb];
        }
    lf.fb = fb;
    lf.L = nb - fb;
    lf.fl = lf.f - fb;
    lf.inv_dx = idx;
    lf.dx = dxb;
    return lf;
}

__device__ inline LaneFreq lane_freq(const SolveLaunch& a, int fc, int lane) { return lane_freq_at(a, fc * 64 + lane); }

// Reciprocals.  FP32: the hardware reciprocal (1 ulp).  FP64: the hardware
// estimate refined by two Newton steps r <- r + r(1 - x r), within about 1 ulp
// (an IEEE division costs several times more and is not needed for 1e-12).
__device__ inline double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return r;
}

// min(max(x, lo), hi) for lo <= hi in one instruction (the compiler forms
// v_med3_i32 only for constant bounds).
__device__ inline int clamp_i32(int x, int lo, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

template <typename T>
__device__ inline T fma_(T a, T b, T c) { return __builtin_fma(a, b, c); }
template <>
__device__ inline float fma_<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ inline T rcp(T x);
template <>
__device__ inline float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ inline double rcp<double>(double x) { return rcp64(x); }

// Running state of one side's elimination (file header).
template <typename T>
struct SweepState {
    T G, Y, r;  // rescaled pivot and right-hand side, r = 1/(1 + a G)
    T a;        // inner optical-depth step of the last row: the outer step of the next
    // fourth-order rows: u_d = (1 - F) u_{d+1} + Z; S (FP64) of the last row's
    // point and of its next point; whether a row met a step beyond the limit
    T F, Z;
    double Sp, Sc;
    bool bad;
};

// Row d of the elimination, given its inner step b and S_d (the outer step is st.a).
template <typename T>
__device__ inline void row(SweepState<T>& st, bool far_end, T b, T S, T I) {
    if (far_end) {
        const T hb = (T)0.5 * b;
        st.G = (T)1 + hb;
        st.r = rcp<T>(fma_<T>(b, st.G, (T)1));
        st.Y = fma_<T>(hb, S, I) * st.r;
    } else {
        const T h = (T)0.5 * (st.a + b);
        st.G = fma_<T>(st.G, st.r, h);
        st.r = rcp<T>(fma_<T>(b, st.G, (T)1));
        st.Y = fma_<T>(h, S, st.Y) * st.r;
    }
    st.a = b;
}

// Row d of the second-order elimination for a point of opacity c whose source the
// next row needs: the row's reciprocal r = 1/D (D = 1 + b G) and 1/c come from one
// reciprocal of their product, q = 1/(D c), r = q c, 1/c = q D (three multiplies
// instead of a second quarter-rate reciprocal; D >= 1 and c > 0, so the product
// neither cancels nor, for opacities below ~1e30, overflows).  Returns 1/c.  The sweep
// starts a side from the state G = 1, r = 1, a = 0, Y = I, on which this generic row
// with the far end's step is the far-end row of `row` (G = 1 + b/2, Y = (b/2 S + I) r),
// and runs it for the first point too, with b = 0: that row leaves G = 1, a = 0 and
// r, Y within an ulp of 1 and I, and yields the first point's 1/c.
template <typename T>
__device__ inline T row_rc(SweepState<T>& st, T b, T S, T c) {
    const T h = (T)0.5 * (st.a + b);
    st.G = fma_<T>(st.G, st.r, h);
    const T D = fma_<T>(b, st.G, (T)1);
    const T q = rcp<T>(D * c);
    st.r = q * c;
    st.Y = fma_<T>(h, S, st.Y) * st.r;
    st.a = b;
    return q * D;
}

// Fourth-order (Hermitian) rows with third-order end rows: the scheme Section
// 2.1 names for the solver (Auer 1976); derived from exactness for quartic u.
// A row d with outer step a, inner step b (toward the origin) reads
//   -A' u_far + (1 + A' + C') u_d - C' u_near = al S_far + (1 - al - ga) S_d + ga S_near,
//   al = w(a, b), ga = w(b, a),  w(x, y) = (x^3 + 2x^2 y - y^3) / (6 x (x+y)^2),
//   A' = 2/(a(a+b)) - al,  C' = 2/(b(a+b)) - ga,
// and the far end (step t to its neighbour) with E = (2/t)(1 + t^2/6):
//   (1 + E + 2/t^2) u_0 - (2/t^2) u_1 = S_0 + E I + (S_1 - S_0)/3.
// The right-hand side is formed as S_d + al (S_far - S_d) + ga (S_near - S_d)
// (al + be + ga = 1) with S = eta/chi and this sum in FP64, rounded once to the
// kernel's precision: for unequal steps one weight grows like the step ratio
// (which reaches 1e3 and more on unstructured lines), so an S rounded to FP32,
// or the literal form be S_d + ga S_near, would carry that factor into u.
// With u_d = (1 - H_d) u_{d+1} + Z_d (H = F/(1+F) of the usual u_d =
// u_{d+1}/(1+F_d) + Z_d) the elimination takes one reciprocal per row:
//   D = 1 + C' + A' H_{d-1},  H_d = (1 + A' H_{d-1}) / D,  Z_d = (R_d + A' Z_{d-1}) / D,
// sums of non-negative terms while A' >= 0 and C' > 0 (steps below about
// 3.46); a row beyond that marks the side bad (reported as an error).
// The weights in the scale-free form: with s = a + b, p = a/s, q = b/s,
//   al = P/(6p), ga = Q/(6q),  P = p^2 (p + 2q) - q^3,  Q = q^2 (q + 2p) - p^3,
//   A' = (12/s^2 - P)/(6p),  C' = (12/s^2 - Q)/(6q),
// so no cube of a step can underflow and three reciprocals give all four.
template <typename T>
struct HermCoef {
    T al, ga, Am, Cp;
};

template <typename T>
__device__ inline HermCoef<T> herm_coef(T a, T b) {
    const T rs = rcp<T>(a + b);
    const T p = a * rs, q = b * rs;
    const T t12 = (T)12 * rs * rs;
    const T P = fma_<T>(p * p, p + (q + q), -(q * q * q));
    const T Q = fma_<T>(q * q, q + (p + p), -(p * p * p));
    const T r6p = rcp<T>((T)6 * p), r6q = rcp<T>((T)6 * q);
    return HermCoef<T>{P * r6p, Q * r6q, (t12 - P) * r6p, (t12 - Q) * r6q};
}

// S = eta/chi in FP64 through the refined reciprocal (within an ulp or two of
// the correctly rounded quotient: the rows' own rounding sensitivity, which the
// parity bar of these rows allows, is larger).
template <typename T>
__device__ inline double src64(T e, T c) { return (double)e * rcp64((double)c); }

// Row d: its inner step b, its own optics (c, e) and the next point's (cn, en).
// The state carries S of the previous row's point (Sp) and of this one (Sc,
// the previous row's next point), so each row forms one new FP64 S.
template <typename T>
__device__ inline void row_h(SweepState<T>& st, bool far_end, T b, T c, T e, T cn, T en, T I) {
    const double Sn = src64<T>(en, cn);
    if (far_end) {
        // (1 + E + K) u_0 - K u_1 = R_0, K = 2/b^2, scaled by b^2/2
        const double S = src64<T>(e, c);
        const T rb = rcp<T>(b);
        const T E = (T)2 * rb * fma_<T>(b * b, (T)(1.0 / 6.0), (T)1);
        const T hk = (T)0.5 * b * b;  // 1/K
        const T F0 = ((T)1 + E) * hk;
        const T R0 = (T)(S + __builtin_fma((double)E, (double)I, (Sn - S) * (1.0 / 3.0)));
        const T rD = rcp<T>((T)1 + F0);
        st.F = F0 * rD;
        st.Z = R0 * hk * rD;
        st.Sc = S;
    } else {
        const double S = st.Sc;
        const HermCoef<T> k = herm_coef<T>(st.a, b);
        st.bad = st.bad || !(k.Am >= (T)0) || !(k.Cp > (T)0);
        const T R = (T)__builtin_fma((double)k.al, st.Sp - S, __builtin_fma((double)k.ga, Sn - S, S));
        const T rD = rcp<T>((T)1 + fma_<T>(k.Am, st.F, k.Cp));
        st.Z = fma_<T>(k.Am, st.Z, R) * rD;
        st.F = fma_<T>(k.Am, st.F, (T)1) * rD;
    }
    st.a = b;
    st.Sp = st.Sc;
    st.Sc = Sn;
}

// u at the origin with the fourth-order rows: each non-empty side's last row
// had the origin as its next point, so its state holds S_o (Sc) and S of its
// last point (Sp).
template <typename T>
__device__ inline T origin_h(bool hm, bool hp, SweepState<T>& m, SweepState<T>& p, T I) {
    if (hm && hp) {
        const double S = m.Sc;
        const HermCoef<T> k = herm_coef<T>(m.a, p.a);
        m.bad = m.bad || !(k.Am >= (T)0) || !(k.Cp > (T)0);
        const T R = (T)__builtin_fma((double)k.al, m.Sp - S, __builtin_fma((double)k.ga, p.Sp - S, S));
        const T den = (T)1 + fma_<T>(k.Am, m.F, k.Cp * p.F);
        return fma_<T>(k.Am, m.Z, fma_<T>(k.Cp, p.Z, R)) * rcp<T>(den);
    }
    if (hm || hp) {
        const SweepState<T>& q = hp ? p : m;
        const double S = q.Sc;
        const T t = q.a, rt_ = rcp<T>(t);
        const T E = (T)2 * rt_ * fma_<T>(t * t, (T)(1.0 / 6.0), (T)1);
        const T K = (T)2 * rt_ * rt_;
        const T R0 = (T)(S + __builtin_fma((double)E, (double)I, (q.Sp - S) * (1.0 / 3.0)));
        return fma_<T>(K, q.Z, R0) * rcp<T>((T)1 + E + K * q.F);
    }
    return I;
}

// A row of the chosen scheme.  SCH 0, second order: the point's S.  SCH 1,
// fourth order: the point's optics and the next point's (cn, en).
template <typename T, int SCH>
__device__ inline void row_s(SweepState<T>& st, bool far_end, T b, T S, T c, T e, T cn, T en, T I) {
    if (SCH == 1) row_h<T>(st, far_end, b, c, e, cn, en, I);
    else row<T>(st, far_end, b, S, I);
}

// u at the origin from the two sides' states (file header).
template <typename T>
__device__ inline T origin_u(bool hm, bool hp, const SweepState<T>& m, const SweepState<T>& p, T S, T I) {
    if (hm && hp) {
        const T h = (T)0.5 * (m.a + p.a);
        return fma_<T>(h, S, m.Y + p.Y) * rcp<T>(h + fma_<T>(m.G, m.r, p.G * p.r));
    }
    if (hm || hp) {
        const SweepState<T>& q = hp ? p : m;
        const T ht = (T)0.5 * q.a;
        return (fma_<T>(ht, S, I) + q.Y) * rcp<T>(fma_<T>(q.G, q.r, (T)1 + ht));
    }
    return I;
}

// Per-wave constants of one item.
struct ItemCtx {
    const char* chi;   // table bases (bytes)
    const char* eta;
    int64_t ld_bytes;  // row stride in bytes
    const int32_t* ids;
    const double* Zr;
    const float* vel;
    double nx, ny, nz, inv_dx0;
    float vox, voy, voz;
    double dtau_rcp;   // adaptive optical-depth increments: 1/dtau_max
    double dv_rcp;     // adaptive velocity sampling: 1/dv_max
    double dx0;        // width of the first block's frequency step
    int64_t row_o;     // the origin's table row offset in bytes
    int max_sub;
};

// ---------------------------------------------------------------- refined lines
// Adaptive velocity sampling (Section 2.1.1) and adaptive optical-depth
// increments (Section 2.1.2, eq. 2) generate extra line points on the fly,
// between consecutive points of a ray list, in registers.
//
// Both split counts are integers decided from floating point, so they are
// decided in FP64 with the oracle's arithmetic: the projected velocities
// p = n.(v - v_o), the shift p/dx (a division), chi' of a point as
// (1-w)((1-t) a0 + t a1) + w((1-t) b0 + t b1) from its table values (a: the
// end point of smaller line coordinate, b: the other; w = 0 for a point of
// the list), lengths ds and ds/m, and the products with the reciprocals of the
// bounds.  The optics that enter the solve are computed in the kernel's
// precision.

// What the FP64 split decision needs of a line point.
template <typename T>
struct Pt64 {
    T a0, a1, b0, b1;  // table values: end points a and b at rows f - k and f - k - 1
    double t, w;       // shift fraction, weight of b
};

template <typename T>
__device__ inline double chi64(const Pt64<T>& p) {
    return (1.0 - p.w) * ((1.0 - p.t) * (double)p.a0 + p.t * (double)p.a1) +
           p.w * ((1.0 - p.t) * (double)p.b0 + p.t * (double)p.b1);
}

// Interval from the far point (chi cf, eta ef, S Sf) to the near point (cn, en)
// of one side: n = ceil(max(chi'_far, chi'_near) ds / dtau_max), clamped to
// 1 .. max_sub; hds is half the interval's length.  When the kernel-precision
// estimate is below 1 - 1e-4 in every lane (it is within a few ulps of the FP64
// value) n is 1 everywhere and the FP64 evaluation is skipped.  The n-1
// interior points interpolate chi' and eta' linearly; rows are emitted far to
// near, each with its inner step, the last being the sub-point next to the near
// point.  `first` marks the far end of the line (its row is the boundary row).
// With the second-order rows (SCH 0) every row whose near point is a line point forms that
// point's 1/chi with the row's reciprocal (row_rc) and the interval returns it; the row into
// the origin (to_origin) is the plain row, a far-end row when it is the line's first.
template <typename T, int SCH>
__device__ inline T near_row(SweepState<T>& st, bool first, T b, T Sf, T cf, T ef, T cn, T en, T I, bool to_origin) {
    if (SCH == 0) {
        if (!to_origin) return row_rc<T>(st, b, Sf, cn);
        row<T>(st, first, b, Sf, I);
        return (T)0;
    }
    row_s<T, SCH>(st, first, b, Sf, cf, ef, cn, en, I);
    return (T)0;
}

template <typename T, int SCH>
__device__ inline T substep_interval(const ItemCtx& c, SweepState<T>& st, bool first, T cf, T ef, T Sf, T cn, T en,
                                     T hds, const Pt64<T>& pf, const Pt64<T>& pn, double ds64, T I, bool to_origin) {
    const T est = (cf > cn ? cf : cn) * (hds + hds) * (T)c.dtau_rcp;
    if (!__builtin_amdgcn_ballot_w64(est > (T)0.9999))
        return near_row<T, SCH>(st, first, (cf + cn) * hds, Sf, cf, ef, cn, en, I, to_origin);
    const double c64f = chi64(pf), c64n = chi64(pn);
    const double cm = c64f > c64n ? c64f : c64n;
    double q = ceil((cm * ds64) * c.dtau_rcp);
    if (q > (double)c.max_sub) q = (double)c.max_sub;
    const int n = q >= 1.0 ? (int)q : 1;  // also 1 for a NaN
    const T rn = rcp<T>((T)n);
    const T hh = hds * rn;  // half a sub-interval
    T cp = cf, ep = ef, Sp = Sf;
    bool fr = first;
    for (int k = 1; __builtin_amdgcn_ballot_w64(k < n); ++k) {
        if (k < n) {
            const T w = (T)k * rn;
            const T ck = fma_<T>(w, cn - cf, cf);
            const T ek = fma_<T>(w, en - ef, ef);
            const T ic = near_row<T, SCH>(st, fr, (cp + ck) * hh, Sp, cp, ep, ck, ek, I, false);
            cp = ck;
            ep = ek;
            if (SCH == 0) Sp = ek * ic;
            fr = false;
        }
    }
    return near_row<T, SCH>(st, fr, (cp + cn) * hh, Sp, cp, ep, cn, en, I, to_origin);
}

// The stream of line points of one side, far to near, after velocity sampling.
template <typename T>
struct Emitter {
    T c, e, S;
    Pt64<T> p;
    bool first = true;  // no row emitted yet: the next one is the boundary row
    bool have = false;
};

// Emit the next line point; the interval from the previous one (half length
// hds, FP64 length ds64) is split by optical depth when that is on.
// (SCH 0: Sn is ignored and formed from the row's reciprocal, the first point's from the
// harmless row of row_rc; the state starts as row_rc describes.)
template <typename T, int SCH>
__device__ inline void emit_point(const ItemCtx& c, SweepState<T>& st, Emitter<T>& em, T cn, T en, T Sn,
                                  const Pt64<T>& pn, T hds, double ds64, T I, bool to_origin) {
    if (em.have) {
        T ic;
        if (c.dtau_rcp > 0.0)
            ic = substep_interval<T, SCH>(c, st, em.first, em.c, em.e, em.S, cn, en, hds, em.p, pn, ds64, I,
                                          to_origin);
        else ic = near_row<T, SCH>(st, em.first, (em.c + cn) * hds, em.S, em.c, em.e, cn, en, I, to_origin);
        if (SCH == 0) Sn = en * ic;
        em.first = false;
    } else if (SCH == 0) {
        Sn = en * row_rc<T>(st, (T)0, (T)0, cn);
    }
    em.c = cn;
    em.e = en;
    em.S = Sn;
    em.p = pn;
    em.have = true;
}

// A list point (real) of the current side, as the refinement needs it.
template <typename T>
struct RealPt {
    T c, e, S;
    Pt64<T> p;
    double dot;   // projected velocity n.(v - v_o)
    int64_t row;  // table row offset in bytes
};

// Interval from real point P (far) to real point C (near), hds / ds64 its half
// and FP64 lengths: velocity sub-points first (m from |p_C - p_P|), each emitted,
// then C itself.  fwd: this side is the +n ray, whose nearer point has the
// smaller line coordinate (so it is the interval's point a).
template <typename T, bool UDX, int SCH>
__device__ inline void real_interval(const ItemCtx& c, SweepState<T>& st, Emitter<T>& em, const RealPt<T>& P,
                                     const RealPt<T>& C, T hds, double ds64, bool fwd, const LaneFreq& lf, T I,
                                     bool to_origin) {
    int m = 1;
    if (c.dv_rcp > 0.0) {
        double q = ceil(fabs(C.dot - P.dot) * c.dv_rcp);
        if (q > (double)c.max_sub) q = (double)c.max_sub;
        m = q >= 1.0 ? (int)q : 1;
        m = __builtin_amdgcn_readfirstlane(m);  // the same in every lane
    }
    if (m == 1) {
        emit_point<T, SCH>(c, st, em, C.c, C.e, C.S, C.p, hds, ds64, I, to_origin);
        return;
    }
    const T hs = hds * rcp<T>((T)m);
    const double ds64s = ds64 / (double)m;
    const RealPt<T>& A = fwd ? C : P;  // the end point of smaller line coordinate
    const RealPt<T>& B = fwd ? P : C;
    const double dx = UDX ? c.dx0 : lf.dx;
    const int lb_bytes = (lf.fb + lf.fl) * (int)sizeof(T);
    const int lo_bytes = lf.fb * (int)sizeof(T);
    const int hi_bytes = (lf.fb + lf.L - 1) * (int)sizeof(T);
    for (int jj = 1; jj < m; ++jj) {  // far to near
        const int jo = fwd ? m - jj : jj;
        const double w = (double)jo / (double)m;
        const double vdot = (1.0 - w) * A.dot + w * B.dot;
        const double delta = vdot / dx;
        const double kf = floor(delta);
        const int k = (int)kf;
        const double t64 = delta - kf;
        const T t = (T)t64;
        const int ks = k * (int)sizeof(T);
        const uint32_t oa = (uint32_t)clamp_i32(lb_bytes - ks, lo_bytes, hi_bytes);
        const uint32_t ob = (uint32_t)clamp_i32(lb_bytes - (int)sizeof(T) - ks, lo_bytes, hi_bytes);
        const T a0 = *(const T*)(c.chi + A.row + oa), a1 = *(const T*)(c.chi + A.row + ob);
        const T b0 = *(const T*)(c.chi + B.row + oa), b1 = *(const T*)(c.chi + B.row + ob);
        const T g0 = *(const T*)(c.eta + A.row + oa), g1 = *(const T*)(c.eta + A.row + ob);
        const T h0 = *(const T*)(c.eta + B.row + oa), h1 = *(const T*)(c.eta + B.row + ob);
        const T wt = (T)w;
        const T xa = fma_<T>(t, a1 - a0, a0), xb = fma_<T>(t, b1 - b0, b0);
        const T ya = fma_<T>(t, g1 - g0, g0), yb = fma_<T>(t, h1 - h0, h0);
        const T cv = fma_<T>(wt, xb - xa, xa);
        const T ev = fma_<T>(wt, yb - ya, ya);
        emit_point<T, SCH>(c, st, em, cv, ev, SCH == 0 ? (T)0 : ev * rcp<T>(cv), Pt64<T>{a0, a1, b0, b1, t64, w},
                           hs, ds64s, I, false);
    }
    emit_point<T, SCH>(c, st, em, C.c, C.e, C.S, C.p, hs, ds64s, I, to_origin);
}

// One side of the line with velocity sampling and/or optical-depth sub-steps
// (the plain sweep below is the same without them).
// Per-point records of the refined sweep in LDS: words 0-1 row offset (bytes),
// 2-3 projected velocity (FP64), 4-5 the FP64 interval length to the previous
// list point, 6 the whole-step shift (uniform dx), 8-9 its FP64 fraction.
constexpr int REF_STAGE_WORDS = 12;

template <typename T, bool MOVING, bool UDX, int SCH>
__device__ inline void sweep_ref(const ItemCtx& c, int64_t base, int n, const LaneFreq& lf, int lane, bool fwd,
                                 T chi_o, T eta_o, T S_o, T I, SweepState<T>& st, uint32_t* stage) {
    Emitter<T> em;
    RealPt<T> prev{};
    T hds_prev = (T)0;
    double ds64_prev = 0.0;
    int done = 0;
    if (SCH == 0) {  // the state before the far end (row_rc)
        st.G = (T)1;
        st.r = (T)1;
        st.a = (T)0;
        st.Y = I;
    }
    const uint32_t lane_off = (uint32_t)lf.f * (uint32_t)sizeof(T);
    const int lb_bytes = (lf.fb + lf.fl) * (int)sizeof(T);
    const int lo_bytes = lf.fb * (int)sizeof(T);
    const int hi_bytes = (lf.fb + lf.L - 1) * (int)sizeof(T);
    for (int hi = n - 1; hi >= 0; hi -= 64) {
        const int cnt = hi + 1 < 64 ? hi + 1 : 64;
        const int e = hi - lane;
        if (lane < cnt) {  // lane j stages the record of entry hi-j
            uint32_t* w = stage + lane * REF_STAGE_WORDS;
            const int q = c.ids[base + e];
            const uint64_t row = (uint64_t)q * (uint64_t)c.ld_bytes;
            const double z = c.Zr[base + e];
            const double zi = e > 0 ? c.Zr[base + e - 1] : 0.0;
            w[0] = (uint32_t)row;
            w[1] = (uint32_t)(row >> 32);
            *(double*)(w + 4) = z - zi;
            double dot = 0.0;
            if (MOVING) {
                const float* vq = c.vel + 3 * (int64_t)q;
                const double dvx = (double)vq[0] - (double)c.vox;
                const double dvy = (double)vq[1] - (double)c.voy;
                const double dvz = (double)vq[2] - (double)c.voz;
                dot = (c.nx * dvx + c.ny * dvy) + c.nz * dvz;
                if (UDX) {  // the same shift in every lane: formed once per point while staging
                    const double delta = dot / c.dx0;
                    const double kf = floor(delta);
                    w[6] = (uint32_t)(int)kf;
                    *(double*)(w + 8) = delta - kf;
                }
            }
            *(double*)(w + 2) = dot;
        }
        __builtin_amdgcn_wave_barrier();
        // the table values of point j are loaded while point j-1 is processed
        struct Fetch {
            int64_t row;
            double dot, ds64, t64;
            T ca, cb, ea, eb;
        };
        auto fetch = [&](int j) {
            const uint32_t* w = stage + j * REF_STAGE_WORDS;
            Fetch f;
            f.row = uni64((int64_t)(((uint64_t)w[1] << 32) | w[0]));
            f.dot = MOVING ? *(const double*)(w + 2) : 0.0;
            f.ds64 = *(const double*)(w + 4);
            f.t64 = 0.0;
            const char* cr = c.chi + f.row;
            const char* er = c.eta + f.row;
            if (MOVING) {
                int k;
                if (UDX) {
                    k = (int)w[6];
                    f.t64 = *(const double*)(w + 8);
                } else {
                    const double delta = f.dot / lf.dx;
                    const double kf = floor(delta);
                    k = (int)kf;
                    f.t64 = delta - kf;
                }
                const int ks = k * (int)sizeof(T);
                const uint32_t oa = (uint32_t)clamp_i32(lb_bytes - ks, lo_bytes, hi_bytes);
                const uint32_t ob = (uint32_t)clamp_i32(lb_bytes - (int)sizeof(T) - ks, lo_bytes, hi_bytes);
                f.ca = *(const T*)(cr + oa);
                f.cb = *(const T*)(cr + ob);
                f.ea = *(const T*)(er + oa);
                f.eb = *(const T*)(er + ob);
            } else {
                f.ca = f.cb = *(const T*)(cr + lane_off);
                f.ea = f.eb = *(const T*)(er + lane_off);
            }
            return f;
        };
        Fetch nxt = fetch(0);
        for (int j = 0; j < cnt; ++j) {
            const Fetch f = nxt;
            if (j + 1 < cnt) nxt = fetch(j + 1);
            const double ds64 = f.ds64;
            RealPt<T> cur;
            cur.row = f.row;
            cur.dot = f.dot;
            if (MOVING) {
                const T t = (T)f.t64;
                cur.c = fma_<T>(t, f.cb - f.ca, f.ca);
                cur.e = fma_<T>(t, f.eb - f.ea, f.ea);
                cur.p = Pt64<T>{f.ca, f.cb, f.ca, f.cb, f.t64, 0.0};
            } else {
                cur.c = f.ca;
                cur.e = f.ea;
                cur.p = Pt64<T>{cur.c, cur.c, cur.c, cur.c, 0.0, 0.0};
            }
            cur.S = SCH == 0 ? (T)0 : cur.e * rcp<T>(cur.c);  // SCH 0: formed with the row (emit_point)
            if (done == 0) emit_point<T, SCH>(c, st, em, cur.c, cur.e, cur.S, cur.p, (T)0, 0.0, I, false);
            else real_interval<T, UDX, SCH>(c, st, em, prev, cur, hds_prev, ds64_prev, fwd, lf, I, false);
            prev = cur;
            ds64_prev = ds64;
            hds_prev = (T)0.5 * (T)ds64;
            ++done;
        }
        __builtin_amdgcn_wave_barrier();  // every lane has read this run before the next is staged
    }
    if (n > 0) {
        RealPt<T> org;
        org.c = chi_o;
        org.e = eta_o;
        org.S = S_o;
        org.p = Pt64<T>{chi_o, chi_o, chi_o, chi_o, 0.0, 0.0};
        org.dot = 0.0;
        org.row = c.row_o;
        real_interval<T, UDX, SCH>(c, st, em, prev, org, hds_prev, ds64_prev, fwd, lf, I, true);
    }
}

// Per-point data of the line points being swept, staged in LDS: 64 records of
// eight 32-bit words per wave.  Words 0-1: table row offset in bytes; with a
// uniform dx, word 2 the whole-step shift in bytes and word 3 (FP32) or 4-5
// (FP64) the fraction t, otherwise words 2-3 the projected velocity (FP64);
// word 4 (FP32) or 6-7 (FP64): ds/2.
constexpr int STAGE_WORDS = 8;

// Eliminate one side of the line (entries base .. base+n-1 of a ray list,
// walked from the far end inwards), up to the origin; on return st holds the
// row next to the origin and st.a the step between that row and the origin.
//
// Staging: for each run of 64 points, lane j computes the record of point
// hi-j (id, ds from the FP64 Z, and with a uniform dx the Doppler shift as
// whole steps + fraction, the same in every lane) and writes it to LDS; the
// elimination then reads one record per point with a broadcast LDS read, so
// the per-point values reach every lane without VALU lane transfers.  SMALL:
// the tables are below 4 GiB, so a lane's address is the table base (scalar)
// plus a 32-bit offset row + its clamped column; otherwise the row offset is
// moved to scalar registers per point.
// GROUP line points have their loads issued together before the recurrence
// consumes them (a tuning parameter: more points in flight per wave against
// more registers, i.e. fewer waves).
template <typename T, bool MOVING, bool UDX, int GROUP, bool SMALL, int SCH>
__device__ inline void sweep(const ItemCtx& c, int64_t base, int n, const LaneFreq& lf, int lane, T chi_o, T eta_o,
                             T I, SweepState<T>& st, uint32_t* stage) {
    T c_prev = (T)0, e_prev = (T)0, S_prev = (T)0, ds_prev = (T)0;
    int done = 0;
    if (SCH == 0) {  // the state before the far end (row_rc)
        st.G = (T)1;
        st.r = (T)1;
        st.a = (T)0;
        st.Y = I;
    }
    const uint32_t lane_off = (uint32_t)lf.f * (uint32_t)sizeof(T);
    // the lane's own frequency and its block's first and last, in bytes
    const int lb_bytes = (lf.fb + lf.fl) * (int)sizeof(T);
    const int lbm_bytes = lb_bytes - (int)sizeof(T);
    const int lo_bytes = lf.fb * (int)sizeof(T);
    const int hi_bytes = (lf.fb + lf.L - 1) * (int)sizeof(T);
    constexpr int T_WORD = sizeof(T) == 4 ? 3 : 4;   // the fraction t
    constexpr int DS_WORD = sizeof(T) == 4 ? 4 : 6;  // ds/2
    for (int hi = n - 1; hi >= 0; hi -= 64) {
        const int cnt = hi + 1 < 64 ? hi + 1 : 64;
        // staging: lane j writes the record of entry hi-j
        const int e = hi - lane;
        if (lane < cnt) {
            uint32_t* w = stage + lane * STAGE_WORDS;
            const int q = c.ids[base + e];
            const uint64_t row = (uint64_t)q * (uint64_t)c.ld_bytes;
            const double z = c.Zr[base + e];
            const double zi = e > 0 ? c.Zr[base + e - 1] : 0.0;
            const T ds = (T)0.5 * (T)(z - zi);  // half the difference of FP64 projections, rounded once
            w[0] = (uint32_t)row;
            w[1] = (uint32_t)(row >> 32);
            if (MOVING) {
                const float* vq = c.vel + 3 * (int64_t)q;
                const double dvx = (double)vq[0] - (double)c.vox;
                const double dvy = (double)vq[1] - (double)c.voy;
                const double dvz = (double)vq[2] - (double)c.voz;
                const double dot = (c.nx * dvx + c.ny * dvy) + c.nz * dvz;
                if (UDX) {
                    const double delta = dot / c.dx0;
                    const double kf = floor(delta);
                    w[2] = (uint32_t)((int)kf * (int)sizeof(T));
                    *(T*)(w + T_WORD) = (T)(delta - kf);
                } else {
                    *(double*)(w + 2) = dot;
                }
            }
            *(T*)(w + DS_WORD) = ds;
        }
        __builtin_amdgcn_wave_barrier();
        // a group of GROUP points: loads first, then the recurrence; FULL groups
        // carry no per-point bounds test, so their loads are issued together
        auto point_group = [&](auto full, int j) {
            constexpr bool FULL = decltype(full)::value;
            T ca[GROUP], cb[GROUP], ea[GROUP], eb[GROUP], tt[GROUP], dsv[GROUP];
#pragma unroll
            for (int g = 0; g < GROUP; ++g) {
                if (FULL || j + g < cnt) {
                    const uint32_t* w = stage + (j + g) * STAGE_WORDS;
                    const uint4 r0 = *(const uint4*)w;  // one broadcast read: row, shift, t
                    dsv[g] = *(const T*)(w + DS_WORD);
                    const char* cr = c.chi;
                    const char* er = c.eta;
                    uint32_t rlo = r0.x;
                    if (!SMALL) {  // the row in scalar registers, the column as the offset
                        const uint64_t row = uni64((int64_t)(((uint64_t)r0.y << 32) | r0.x));
                        cr += row;
                        er += row;
                        rlo = 0;
                    }
                    if (MOVING) {
                        int ks;
                        T t;
                        if (UDX) {
                            ks = (int)r0.z;
                            t = *(const T*)(w + T_WORD);
                        } else {  // per-lane block widths: the shift as the oracle forms it, a division
                            const double delta = __builtin_bit_cast(double, (((uint64_t)r0.w << 32) | r0.z)) / lf.dx;
                            const double kf = floor(delta);
                            ks = (int)kf * (int)sizeof(T);
                            t = (T)(delta - kf);
                        }
                        // byte offsets of rows fl - k and fl - k - 1, clamped to the block
                        const uint32_t oa = rlo + (uint32_t)clamp_i32(lb_bytes - ks, lo_bytes, hi_bytes);
                        const uint32_t ob = rlo + (uint32_t)clamp_i32(lbm_bytes - ks, lo_bytes, hi_bytes);
                        ca[g] = *(const T*)(cr + oa);
                        cb[g] = *(const T*)(cr + ob);
                        ea[g] = *(const T*)(er + oa);
                        eb[g] = *(const T*)(er + ob);
                        tt[g] = t;
                    } else {
                        const uint32_t o = rlo + lane_off;
                        ca[g] = *(const T*)(cr + o);
                        ea[g] = *(const T*)(er + o);
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < GROUP; ++g) {
                if (FULL || j + g < cnt) {
                    T cc, et;
                    if (MOVING) {
                        cc = fma_<T>(tt[g], cb[g] - ca[g], ca[g]);
                        et = fma_<T>(tt[g], eb[g] - ea[g], ea[g]);
                    } else {
                        cc = ca[g];
                        et = ea[g];
                    }
                    if (SCH == 0) {
                        // the row and this point's 1/chi from one reciprocal; at the first point
                        // c_prev and ds_prev are 0, so dt = 0 (see row_rc)
                        const T dt = (c_prev + cc) * ds_prev;  // ds_prev holds ds/2
                        S_prev = et * row_rc<T>(st, dt, S_prev, cc);
                    } else if (done > 0) {
                        const T dt = (c_prev + cc) * ds_prev;
                        row_s<T, SCH>(st, done == 1, dt, S_prev, c_prev, e_prev, cc, et, I);
                    }
                    c_prev = cc;
                    e_prev = et;
                    ds_prev = dsv[g];
                    ++done;
                }
            }
        };
        int j = 0;
        for (; j + GROUP <= cnt; j += GROUP) point_group(std::true_type{}, j);
        if (j < cnt) point_group(std::false_type{}, j);
        __builtin_amdgcn_wave_barrier();  // every lane has read this run before the next is staged
    }
    if (n > 0) {
        const T dt = (c_prev + chi_o) * ds_prev;
        row_s<T, SCH>(st, n == 1, dt, S_prev, c_prev, e_prev, chi_o, eta_o, I);
    }
}

// ---------------------------------------------------------------- packed half waves
//
// Between 65 and 96 frequencies a pair needs a full wave for its first 64 and half a wave
// for the rest.  The second-chunk items of pairs r and r+1 (r even) share one wave: lanes
// 0-31 take pair r's frequencies 64..F-1, lanes 32-63 those of pair r+1, each half walking
// its own line, and the item of pair r+1 is left empty.  The halves stage their points 32
// at a time, each into its own half of the wave's LDS records, and run the elimination
// together for the longer of the two runs (lanes past the end of their own line are
// masked).  Second-order rows on unrefined lines, tables below 4 GiB (32-bit row offsets);
// the arithmetic of every lane is that of `sweep`, so u is the same bit for bit.
template <typename T, bool MOVING, bool UDX, int GROUP>
__device__ inline void sweep_half(const ItemCtx& c, double nx, double ny, double nz, int64_t base, int n,
                                  const LaneFreq& lf, int lane, T chi_o, T I, SweepState<T>& st,
                                  uint32_t* stage) {
    const int hl = lane & 31;
    uint32_t* my = stage + (lane >> 5) * 32 * STAGE_WORDS;
    T c_prev = (T)0, S_prev = (T)0, ds_prev = (T)0;
    st.G = (T)1;  // the state before the far end (row_rc)
    st.r = (T)1;
    st.a = (T)0;
    st.Y = I;
    const uint32_t lane_off = (uint32_t)lf.f * (uint32_t)sizeof(T);
    const int lb_bytes = (lf.fb + lf.fl) * (int)sizeof(T);
    const int lbm_bytes = lb_bytes - (int)sizeof(T);
    const int lo_bytes = lf.fb * (int)sizeof(T);
    const int hi_bytes = (lf.fb + lf.L - 1) * (int)sizeof(T);
    constexpr int T_WORD = sizeof(T) == 4 ? 3 : 4;
    constexpr int DS_WORD = sizeof(T) == 4 ? 4 : 6;
    const int n0 = __builtin_amdgcn_readlane(n, 0), n1 = __builtin_amdgcn_readlane(n, 32);
    const int n_max = n0 > n1 ? n0 : n1;
    for (int run0 = 0; run0 < n_max; run0 += 32) {
        const int hi = n - 1 - run0;                        // this half's newest entry of the run
        const int cnt = hi + 1 < 32 ? (hi + 1 > 0 ? hi + 1 : 0) : 32;  // this half's points in the run
        const int cnt_max = n_max - run0 < 32 ? n_max - run0 : 32;
        if (hl < cnt) {  // lane hl of a half stages entry hi - hl of its own line
            const int e = hi - hl;
            uint32_t* w = my + hl * STAGE_WORDS;
            const int q = c.ids[base + e];
            const uint64_t row = (uint64_t)q * (uint64_t)c.ld_bytes;
            const double z = c.Zr[base + e];
            const double zi = e > 0 ? c.Zr[base + e - 1] : 0.0;
            const T ds = (T)0.5 * (T)(z - zi);
            w[0] = (uint32_t)row;
            w[1] = (uint32_t)(row >> 32);
            if (MOVING) {
                const float* vq = c.vel + 3 * (int64_t)q;
                const double dvx = (double)vq[0] - (double)c.vox;
                const double dvy = (double)vq[1] - (double)c.voy;
                const double dvz = (double)vq[2] - (double)c.voz;
                const double dot = (nx * dvx + ny * dvy) + nz * dvz;
                if (UDX) {
                    const double delta = dot / c.dx0;
                    const double kf = floor(delta);
                    w[2] = (uint32_t)((int)kf * (int)sizeof(T));
                    *(T*)(w + T_WORD) = (T)(delta - kf);
                } else {
                    *(double*)(w + 2) = dot;
                }
            }
            *(T*)(w + DS_WORD) = ds;
        }
        __builtin_amdgcn_wave_barrier();
        const int c0 = __builtin_amdgcn_readlane(cnt, 0), c1 = __builtin_amdgcn_readlane(cnt, 32);
        const int cnt_min = c0 < c1 ? c0 : c1;  // points both halves have in this run
        // a group of GROUP points per lane: loads first, then the recurrence; groups inside both
        // halves' runs (FULL) carry no per-point test, the rest mask the lanes past their run
        auto half_group = [&](auto full, int j0) {
            constexpr bool FULL = decltype(full)::value;
            T ca[GROUP], cb[GROUP], ea[GROUP], eb[GROUP], tt[GROUP], dsv[GROUP];
#pragma unroll
            for (int g = 0; g < GROUP; ++g) {
                if (FULL || j0 + g < cnt) {
                    const uint32_t* w = my + (j0 + g) * STAGE_WORDS;
                    const uint4 r0 = *(const uint4*)w;
                    dsv[g] = *(const T*)(w + DS_WORD);
                    const uint32_t rlo = r0.x;
                    if (MOVING) {
                        int ks;
                        T t;
                        if (UDX) {
                            ks = (int)r0.z;
                            t = *(const T*)(w + T_WORD);
                        } else {
                            const double delta = __builtin_bit_cast(double, (((uint64_t)r0.w << 32) | r0.z)) / lf.dx;
                            const double kf = floor(delta);
                            ks = (int)kf * (int)sizeof(T);
                            t = (T)(delta - kf);
                        }
                        const uint32_t oa = rlo + (uint32_t)clamp_i32(lb_bytes - ks, lo_bytes, hi_bytes);
                        const uint32_t ob = rlo + (uint32_t)clamp_i32(lbm_bytes - ks, lo_bytes, hi_bytes);
                        ca[g] = *(const T*)(c.chi + oa);
                        cb[g] = *(const T*)(c.chi + ob);
                        ea[g] = *(const T*)(c.eta + oa);
                        eb[g] = *(const T*)(c.eta + ob);
                        tt[g] = t;
                    } else {
                        ca[g] = *(const T*)(c.chi + rlo + lane_off);
                        ea[g] = *(const T*)(c.eta + rlo + lane_off);
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < GROUP; ++g) {
                if (FULL || j0 + g < cnt) {
                    T cc, et;
                    if (MOVING) {
                        cc = fma_<T>(tt[g], cb[g] - ca[g], ca[g]);
                        et = fma_<T>(tt[g], eb[g] - ea[g], ea[g]);
                    } else {
                        cc = ca[g];
                        et = ea[g];
                    }
                    const T dt = (c_prev + cc) * ds_prev;
                    S_prev = et * row_rc<T>(st, dt, S_prev, cc);
                    c_prev = cc;
                    ds_prev = dsv[g];
                }
            }
        };
        int j0 = 0;
        for (; j0 + GROUP <= cnt_min; j0 += GROUP) half_group(std::true_type{}, j0);
        for (; j0 < cnt_max; j0 += GROUP) half_group(std::false_type{}, j0);
        __builtin_amdgcn_wave_barrier();  // every lane has read this run before the next is staged
    }
    if (n > 0) row<T>(st, n == 1, (c_prev + chi_o) * ds_prev, S_prev, I);
}

// The packed item of pairs r, r+1 (r even), frequencies 64.. of each (see sweep_half).
template <typename T, bool MOVING, bool UDX, int GROUP>
__device__ inline void solve_item_half(const SolveLaunch& a, int64_t oi, int64_t r, int64_t o, int lane,
                                       uint32_t* stage) {
    const int64_t rh = r + (lane >> 5);
    const LaneFreq lf = lane_freq_at(a, 64 + (lane & 31));
    const int64_t slot_p = oi * 2 * a.R + 2 * rh;
    const int64_t bp = a.ray_off[slot_p], bm = a.ray_off[slot_p + 1], be = a.ray_off[slot_p + 2];
    const int np = (int)(bm - bp), nm = (int)(be - bm);
    ItemCtx c;
    c.chi = (const char*)a.chi;
    c.eta = (const char*)a.eta;
    c.ld_bytes = a.ld * (int64_t)sizeof(T);
    c.ids = a.ray_ids;
    c.Zr = a.ray_Z;
    c.vel = a.vel;
    const double* dv = a.dirs + 3 * ((a.per_origin ? oi * a.R : 0) + rh);
    const double nx = dv[0], ny = dv[1], nz = dv[2];
    c.nx = c.ny = c.nz = 0.0;
    c.inv_dx0 = a.inv_dx[0];
    c.dx0 = a.dx[0];
    c.vox = c.voy = c.voz = 0.f;
    if (MOVING) {
        c.vox = a.vel[3 * o];
        c.voy = a.vel[3 * o + 1];
        c.voz = a.vel[3 * o + 2];
    }
    c.dtau_rcp = 0.0;
    c.dv_rcp = 0.0;
    c.max_sub = a.max_sub;
    c.row_o = o * c.ld_bytes;
    const T I = (T)a.I_bc[lf.f];
    const T chi_o = ((const T*)a.chi)[o * a.ld + lf.f];
    const T eta_o = ((const T*)a.eta)[o * a.ld + lf.f];
    const T S_o = eta_o * rcp<T>(chi_o);
    SweepState<T> m{}, p{};
    sweep_half<T, MOVING, UDX, GROUP>(c, nx, ny, nz, bm, nm, lf, lane, chi_o, I, m, stage);
    sweep_half<T, MOVING, UDX, GROUP>(c, nx, ny, nz, bp, np, lf, lane, chi_o, I, p, stage);
    const T u = origin_u<T>(nm > 0, np > 0, m, p, S_o, I);
    if (lf.active) {
        ((T*)a.u)[(oi * a.R + rh) * a.F + lf.f] = u;
        if (!(u == u) || u - u != (T)0) atomicOr(a.err, ERRBIT_NONFINITE);
    }
}

template <typename T, bool MOVING, bool UDX, int GROUP, bool REF, int SCH, bool PACK>
__device__ inline void solve_item(const SolveLaunch& a, int64_t w, int nfc, int lane, uint32_t* stage) {
    // w is the same in every lane of the wave
    w = uni64(w);
    const int fc = (int)(w % nfc);
    const int64_t pr = w / nfc;
    const int64_t r = pr % a.R;
    const int64_t oi = pr / a.R;
    const int64_t o = a.origins ? (int64_t)uni(a.origins[oi]) : oi;
    if (o < 0 || o >= a.P) {
        if (lane == 0) atomicOr(a.err, ERRBIT_ORIGIN);
        return;
    }
    if (PACK && fc == 1) {  // launched only for 65..96 frequencies, an even pair count and small tables
        if ((r & 1) == 0) solve_item_half<T, MOVING, UDX, GROUP>(a, oi, r, o, lane, stage);
        return;  // odd pairs: done by the even pair's wave
    }
    const LaneFreq lf = lane_freq(a, fc, lane);
    const int64_t slot_p = oi * 2 * a.R + 2 * r;
    const int64_t bp = uni64(a.ray_off[slot_p]), bm = uni64(a.ray_off[slot_p + 1]);
    const int64_t be = uni64(a.ray_off[slot_p + 2]);
    const int np = (int)(bm - bp), nm = (int)(be - bm);
    ItemCtx c;
    c.chi = (const char*)a.chi;
    c.eta = (const char*)a.eta;
    c.ld_bytes = a.ld * (int64_t)sizeof(T);
    c.ids = a.ray_ids;
    c.Zr = a.ray_Z;
    c.vel = a.vel;
    const double* dv = a.dirs + 3 * ((a.per_origin ? oi * a.R : 0) + r);
    c.nx = dv[0];
    c.ny = dv[1];
    c.nz = dv[2];
    c.inv_dx0 = a.inv_dx[0];
    c.dx0 = a.dx[0];
    c.vox = c.voy = c.voz = 0.f;
    if (MOVING) {
        c.vox = a.vel[3 * o];
        c.voy = a.vel[3 * o + 1];
        c.voz = a.vel[3 * o + 2];
    }
    c.dtau_rcp = a.dtau_max_rcp;
    c.dv_rcp = a.dv_max_rcp;
    c.max_sub = a.max_sub;
    c.row_o = o * c.ld_bytes;
    const T I = (T)a.I_bc[lf.f];
    const T chi_o = ((const T*)a.chi)[o * a.ld + lf.f];
    const T eta_o = ((const T*)a.eta)[o * a.ld + lf.f];
    const T S_o = eta_o * rcp<T>(chi_o);
    SweepState<T> m{}, p{};
    if (REF) {
        sweep_ref<T, MOVING, UDX, SCH>(c, bm, nm, lf, lane, false, chi_o, eta_o, S_o, I, m, stage);
        sweep_ref<T, MOVING, UDX, SCH>(c, bp, np, lf, lane, true, chi_o, eta_o, S_o, I, p, stage);
    } else {
        if (a.small_tables) {
            sweep<T, MOVING, UDX, GROUP, true, SCH>(c, bm, nm, lf, lane, chi_o, eta_o, I, m, stage);
            sweep<T, MOVING, UDX, GROUP, true, SCH>(c, bp, np, lf, lane, chi_o, eta_o, I, p, stage);
        } else {
            sweep<T, MOVING, UDX, GROUP, false, SCH>(c, bm, nm, lf, lane, chi_o, eta_o, I, m, stage);
            sweep<T, MOVING, UDX, GROUP, false, SCH>(c, bp, np, lf, lane, chi_o, eta_o, I, p, stage);
        }
    }
    T u;
    if (SCH == 1) {
        u = origin_h<T>(nm > 0, np > 0, m, p, I);
        if (m.bad || p.bad) {  // a row beyond the step limit: no trustworthy u
            u = (T)NAN;
            if (lf.active) atomicOr(a.err, ERRBIT_STEP);
        }
    } else {
        u = origin_u<T>(nm > 0, np > 0, m, p, S_o, I);
    }
    if (lf.active) {
        ((T*)a.u)[(oi * a.R + r) * a.F + lf.f] = u;
        if (!(u == u) || u - u != (T)0) atomicOr(a.err, ERRBIT_NONFINITE);
    }
}

// Waves per SIMD the direct sweep is compiled for: the FP32 second-order sweep with
// load groups of 4 and one frequency spacing fits 64 VGPRs (one spilled register), so
// 8 waves share a SIMD and hide more of the table loads' latency (on the 64-cloud batch
// 396 ms against 407 at the 7 waves its registers would otherwise allow); its packed
// half-wave variant fits 80 (6 waves, two spilled; the 507k-leaf octree 747 ms against
// 762 with groups of 8 at 4 waves).  The refined sweeps take the bounds below; the
// others keep the compiler's choice (held to 64 registers they spill heavily).
template <typename T, bool UDX, int GROUP, bool REF, int SCH, bool PACK>
constexpr int solve_direct_waves() {
    if (!UDX || GROUP != 4) return 1;
    // refined lines (measured on the 50k wind at dtau_max = 1, spills 0): FP32 second-order rows at 5 waves
    // (39.7 -> 38.6 ms; 6 waves 47.1), fourth-order at 4 (70.8 -> 59.6 ms), FP64 at 3 (78.9 -> 59.1 and
    // 113.5 -> 94.2 ms); the plain FP64 sweep keeps the compiler's choice (43.3 ms against 44.4 at 5 waves)
    if (REF) return sizeof(T) == 4 ? (SCH == 0 ? 5 : 4) : 3;
    return (sizeof(T) == 4 && SCH == 0) ? (PACK ? 6 : 8) : 1;
}

template <typename T, bool MOVING, bool UDX, int GROUP, bool REF, int SCH, bool PACK>
__global__ __launch_bounds__(SOLVE_BLOCK, (solve_direct_waves<T, UDX, GROUP, REF, SCH, PACK>())) void k_solve_direct(
    const SolveLaunch a) {
    constexpr int WORDS = REF ? REF_STAGE_WORDS : STAGE_WORDS;
    __shared__ uint32_t stage_all[WAVES_PER_BLOCK * 64 * WORDS];
    uint32_t* stage = stage_all + (threadIdx.x >> 6) * 64 * WORDS;
    const int lane = threadIdx.x & 63;
    const int nfc = (a.F + 63) / 64;
    const int64_t n_items = a.n_origins * a.R * nfc;
    const int64_t nb = (n_items + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    for (int64_t blk = xcd_block(blockIdx.x, gridDim.x, a.n_xcd, XCD_RUN_SWEEP); blk < nb; blk += gridDim.x) {
        const int64_t it = blk * WAVES_PER_BLOCK + (threadIdx.x >> 6);
        if (it >= n_items) continue;
        int64_t w;
        if (a.order) {  // direction-major over spatially ordered origins (each pair's own order when given)
            const int64_t rc = it / a.n_origins;
            const int64_t q = it - rc * a.n_origins;
            const int64_t oi = a.pair_order ? a.pair_order[(rc / nfc) * a.n_origins + q] : a.order[q];
            w = oi * a.R * nfc + rc;  // rc = r * nfc + chunk
        } else {
            w = a.items ? (int64_t)a.items[it] : it;
        }
        solve_item<T, MOVING, UDX, GROUP, REF, SCH, PACK>(a, w, nfc, lane, stage);
    }
}

// Persistent variant: a fixed grid of waves drains the item queue; each wave
// takes the next PERSIST_CHUNK items with one atomic (one counter shared by
// every wave: an atomic per item serialised the queue) and exits when the
// queue is empty, so every wave reaches the end.
template <typename T, bool MOVING, bool UDX, int GROUP, bool REF, int SCH, bool PACK>
__global__ __launch_bounds__(SOLVE_BLOCK) void k_solve_persist(const SolveLaunch a) {
    constexpr int WORDS = REF ? REF_STAGE_WORDS : STAGE_WORDS;
    __shared__ uint32_t stage_all[WAVES_PER_BLOCK * 64 * WORDS];
    uint32_t* stage = stage_all + (threadIdx.x >> 6) * 64 * WORDS;
    const int lane = threadIdx.x & 63;
    const int nfc = (a.F + 63) / 64;
    const int64_t n_items = a.n_origins * a.R * nfc;
    for (;;) {
        int it0 = 0;
        if (lane == 0) it0 = atomicAdd(a.queue, PERSIST_CHUNK);
        it0 = __builtin_amdgcn_readfirstlane(it0);
        if ((int64_t)it0 >= n_items) break;
        const int64_t end = (int64_t)it0 + PERSIST_CHUNK < n_items ? (int64_t)it0 + PERSIST_CHUNK : n_items;
        for (int64_t it = it0; it < end; ++it) {
            const int64_t w = a.items ? (int64_t)a.items[it] : it;
            solve_item<T, MOVING, UDX, GROUP, REF, SCH, PACK>(a, w, nfc, lane, stage);
        }
    }
}

// J[o][f] = sum over pairs, ascending, of w2_r u_r[f] (eq. 3, eq. 4).
template <typename T>
__global__ __launch_bounds__(256) void k_reduce(const SolveLaunch a) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.n_origins * a.F;
         i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t oi = i / a.F;
    const int f = (int)(i - oi * a.F);
    const T* __restrict__ u = (const T*)a.u + oi * a.R * a.F + f;
    const double* __restrict__ w2 = a.w2 + (a.per_origin ? oi * a.R : 0);
    T acc = (T)0;
    for (int64_t r = 0; r < a.R; ++r) acc += (T)w2[r] * u[r * a.F];
    ((T*)a.J)[i] = acc;
    }
}

// ---------------------------------------------------------------- length binning
// Bin b holds pairs whose line length N = n_- + n_+ + 1 has floor(k log2 N) = b,
// k = bins_per_octave (default 4: quarter-octave bins; the last bin open-ended).  Items are laid out bin by
// bin, longest lines first, so the persistent grid starts the long lines early
// and finishes on short ones.  With a spatial order of the origins (plans), the
// pairs are visited direction by direction over that order, so inside each bin
// consecutive items are neighbouring origins along one direction and share
// table rows in L2, as in the spatial schedule.
__device__ inline int64_t bin_pair(const SolveLaunch& a, int64_t t) {
    if (!a.order) return t;
    const int64_t rc = t / a.n_origins;
    return (int64_t)a.order[t - rc * a.n_origins] * a.R + rc;
}

__device__ inline int bin_of(int64_t N, int n_bins, int per_octave) {
    int b = 0;
    double x = (double)N;
    b = (int)floor((double)per_octave * log2(x));
    if (b < 0) b = 0;
    if (b > n_bins - 1) b = n_bins - 1;
    return b;
}

// Block-local histograms in LDS; one global atomic per non-empty bin per block.
constexpr int MAX_BINS = 128;

__global__ __launch_bounds__(256) void k_bin_count(const SolveLaunch a) {
    __shared__ int h[MAX_BINS];
    for (int i = threadIdx.x; i < a.n_bins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < a.n_origins * a.R) {
        const int64_t s = 2 * bin_pair(a, t);  // slot of the +ray: origin*2R + 2r = 2*(origin*R + r)
        const int64_t N = a.ray_off[s + 2] - a.ray_off[s] + 1;
        atomicAdd(&h[bin_of(N, a.n_bins, a.bins_per_octave)], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.n_bins; i += blockDim.x)
        if (h[i]) atomicAdd(&a.bin_counts[i], h[i]);
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
    __shared__ int h[MAX_BINS];
    __shared__ int base[MAX_BINS];
    for (int i = threadIdx.x; i < a.n_bins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool live = t < a.n_origins * a.R;
    const int64_t p = live ? bin_pair(a, t) : 0;
    int b = 0, local = 0;
    if (live) {
        const int64_t s = 2 * p;
        const int64_t N = a.ray_off[s + 2] - a.ray_off[s] + 1;
        b = bin_of(N, a.n_bins, a.bins_per_octave);
        local = atomicAdd(&h[b], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.n_bins; i += blockDim.x)
        base[i] = h[i] ? atomicAdd(&a.bin_cursor[i], h[i]) : 0;
    __syncthreads();
    if (live) {
        const int nfc = (a.F + 63) / 64;
        const int pos = base[b] + local;
        for (int c = 0; c < nfc; ++c) items[(int64_t)pos * nfc + c] = (int32_t)(p * nfc + c);
    }
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

template <typename T, int G, bool REF, int SCH, bool PACK>
static void solve_dispatch_g(const SolveLaunch& a, bool persist, dim3 grid, hipStream_t s) {
    const bool moving = a.vel != nullptr;
    // the shift of a point is lane-independent when every block has the same dx
    bool udx = true;
    for (int b = 1; b < a.n_blocks; ++b) udx = udx && (a.inv_dx[b] == a.inv_dx[0]);
#define RT_LAUNCH(K, MV, U) hipLaunchKernelGGL((K<T, MV, U, G, REF, SCH, PACK>), grid, dim3(SOLVE_BLOCK), 0, s, a)
    if (persist) {
        if (moving && udx) RT_LAUNCH(k_solve_persist, true, true);
        else if (moving) RT_LAUNCH(k_solve_persist, true, false);
        else RT_LAUNCH(k_solve_persist, false, true);
    } else {
        if (moving && udx) RT_LAUNCH(k_solve_direct, true, true);
        else if (moving) RT_LAUNCH(k_solve_direct, true, false);
        else RT_LAUNCH(k_solve_direct, false, true);
    }
#undef RT_LAUNCH
}

template <typename T>
static void solve_dispatch(const SolveLaunch& a, bool persist, dim3 grid, hipStream_t s) {
    // refined lines (velocity sampling, optical-depth sub-steps) take their own sweep
    const bool ref = a.dtau_max_rcp > 0.0 || a.dv_max_rcp > 0.0;
    // 65..96 frequencies: the second chunks of two pairs share a wave (solve_item_half)
    const bool pack = a.F > 64 && a.F <= 96 && (a.R & 1) == 0 && a.small_tables;
    if (a.scheme == RT_SCHEME_HERMITE) {  // fourth-order rows: one load group size
        if (ref) solve_dispatch_g<T, 4, true, 1, false>(a, persist, grid, s);
        else solve_dispatch_g<T, 4, false, 1, false>(a, persist, grid, s);
    } else if (ref) {
        solve_dispatch_g<T, 4, true, 0, false>(a, persist, grid, s);
    } else if (a.group == 4) {
        if (pack) solve_dispatch_g<T, 4, false, 0, true>(a, persist, grid, s);
        else solve_dispatch_g<T, 4, false, 0, false>(a, persist, grid, s);
    } else {
        if (pack) solve_dispatch_g<T, 8, false, 0, true>(a, persist, grid, s);
        else solve_dispatch_g<T, 8, false, 0, false>(a, persist, grid, s);
    }
}

hipError_t launch_solve(const SolveLaunch& a, int precision, hipStream_t s) {
    const int64_t n_items = solve_items(a);
    if (n_items == 0) return hipSuccess;
    const bool persist = a.schedule == RT_SCHED_BINNED;
    dim3 grid = persist ? dim3((unsigned)((a.grid_waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK))
                        : dim3(capped_blocks((n_items + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK));
    if (precision == RT_F64) solve_dispatch<double>(a, persist, grid, s);
    else solve_dispatch<float>(a, persist, grid, s);
    return hipGetLastError();
}

hipError_t launch_reduce(const SolveLaunch& a, int precision, hipStream_t s) {
    const int64_t n = a.n_origins * a.F;
    if (n == 0) return hipSuccess;
    if (precision == RT_F64)
        hipLaunchKernelGGL(k_reduce<double>, dim3(capped_blocks((n + 255) / 256)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_reduce<float>, dim3(capped_blocks((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace rt
