// Host-side HEALPix ring-scheme tables (Gorski et al. 2005; Section 2.1.3 of the
// paper uses its equal-area pixels, 12*4^l at level l, and its nested hierarchy).
//
// Pixel centres are evaluated with IEEE double arithmetic and the C library's
// cos/sin, in a fixed operation order (no FMA contraction):
//   north cap ring i (pixel j = 1..4i in the ring):  z = 1 - i^2/(3 nside^2),
//                                                     phi = (2j-1) pi / (4i)
//   belt ring i (k = 0..4nside-1, s = (i-nside+1) mod 2):
//                                                     z = 2(2nside-i)/(3nside),
//                                                     phi = (2k+s) pi / (4nside)
//   south cap: mirror of the north cap (z negated), ring 4nside-i
//   vector = (st cos phi, st sin phi, z) with st = sqrt((1-z)(1+z)).
// Antipodes are an exact integer map: ring i <-> ring 4nside-i, half a turn
// along the ring.
#include <cmath>
#include <cstdint>

#include "rt_internal.h"

#pragma clang fp contract(off)

namespace rt {

namespace {

struct RingPos {
    int64_t ring;   // 1 .. 4nside-1 from the north pole
    int64_t first;  // index of the ring's first pixel
    int64_t len;    // pixels in the ring
    int64_t k;      // 0-based position along the ring
};

int64_t int_sqrt(int64_t v) {
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

RingPos locate(int64_t nside, int64_t p) {
    const int64_t npix = 12 * nside * nside;
    const int64_t ncap = 2 * nside * (nside - 1);
    RingPos rp;
    if (p < ncap) {
        int64_t i = (1 + int_sqrt(1 + 2 * p)) >> 1;
        rp.ring = i;
        rp.first = 2 * i * (i - 1);
        rp.len = 4 * i;
    } else if (p < npix - ncap) {
        int64_t i = (p - ncap) / (4 * nside) + nside;
        rp.ring = i;
        rp.first = ncap + (i - nside) * 4 * nside;
        rp.len = 4 * nside;
    } else {
        int64_t q = npix - p;
        int64_t i = (1 + int_sqrt(2 * q - 1)) >> 1;  // ring counted from the south pole
        rp.ring = 4 * nside - i;
        rp.first = npix - 2 * i * (i + 1);
        rp.len = 4 * i;
    }
    rp.k = p - rp.first;
    return rp;
}

}  // namespace

void hp_centre(int64_t nside, int64_t p, double v[3], int64_t* ring) {
    RingPos rp = locate(nside, p);
    double z, phi;
    if (rp.ring < nside) {
        int64_t i = rp.ring, j = rp.k + 1;
        z = 1.0 - (double)(i * i) / (double)(3 * nside * nside);
        phi = (double)(2 * j - 1) * M_PI / (double)(4 * i);
    } else if (rp.ring <= 3 * nside) {
        int64_t i = rp.ring, k = rp.k;
        int64_t s = (i - nside + 1) & 1;
        z = (double)(2 * (2 * nside - i)) / (double)(3 * nside);
        phi = (double)(2 * k + s) * M_PI / (double)(4 * nside);
    } else {
        int64_t i = 4 * nside - rp.ring, j = rp.k + 1;
        z = -(1.0 - (double)(i * i) / (double)(3 * nside * nside));
        phi = (double)(2 * j - 1) * M_PI / (double)(4 * i);
    }
    double st = std::sqrt((1.0 - z) * (1.0 + z));
    v[0] = st * std::cos(phi);
    v[1] = st * std::sin(phi);
    v[2] = z;
    if (ring) *ring = rp.ring;
}

int64_t hp_antipode(int64_t nside, int64_t p) {
    RingPos rp = locate(nside, p);
    const int64_t npix = 12 * nside * nside;
    // The mirror ring has the same length; its pixels are numbered in the same
    // azimuthal order, so half a turn is len/2 positions along it.
    int64_t ring2 = 4 * nside - rp.ring;
    int64_t first2;
    if (ring2 < nside) {
        first2 = 2 * ring2 * (ring2 - 1);
    } else if (ring2 <= 3 * nside) {
        first2 = 2 * nside * (nside - 1) + (ring2 - nside) * 4 * nside;
    } else {
        int64_t i = 4 * nside - ring2;
        first2 = npix - 2 * i * (i + 1);
    }
    return first2 + (rp.k + rp.len / 2) % rp.len;
}

}  // namespace rt
