// Ray tracing through the neighbour graph (Section 2.1, Fig. 2) and the
// device-wide scan that turns ray lengths into list offsets.
//
// From the current point a ray takes the forward neighbour (projection on the
// ray axis strictly beyond the current one) that lies closest to the axis,
// equal distances going to the smaller point id.  The
// geometry is IEEE FP64 in a fixed operation order, the fused multiply-adds
// written out and nothing else contracted (this file is compiled with
// -ffp-contract=off as well): Z = fma(R.z, d.z, fma(R.y, d.y, R.x d.x)),
// q = fma(-Z, d, R) per axis, D = fma(q.z, q.z, fma(q.y, q.y, q.x q.x)).  Every
// list is bit-identical to any other evaluation of the same rule.
//
// Data layout: neighbour records {x, y, z, row start, degree} (32 bytes, two
// 16-byte loads) in CSR order with each row sorted by neighbour id, the ids in
// a parallel array, and a per-point {row start, degree} table, all built once
// per model, so a step reads one record per neighbour instead of an index, a
// position and the next row's offsets; the lanes walking a ray (4 by default)
// read a point's whole row (~15 records, ~500 contiguous bytes) per step.  The walk's loads are
// limited by the vector memory instructions the L1 path serves per clock, so
// a record is two loads, and a chosen neighbour's id is read only when its
// list entry is stored.  The tables of a 50k-point Delaunay mesh (~28 MB)
// stay in the Infinity cache.
#include "rt_internal.h"

#pragma clang fp contract(off)

namespace rt {

namespace {

constexpr int TRACE_BLOCK = 256;

// The records' rows are laid out in the order `lay` (a permutation of the points; NULL:
// point order): the row of point lay[q] is the q-th row in memory.  Degrees in that order:
__global__ __launch_bounds__(256) void k_layout_deg(const int64_t* __restrict__ off, const int32_t* __restrict__ lay,
                                                     int64_t P, int32_t* __restrict__ deg) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P) return;
    const int64_t p = lay ? (int64_t)lay[q] : q;
    deg[q] = (int32_t)(off[p + 1] - off[p]);
}

// rows[lay[q]] = {start of the q-th row (scanned degrees), degree}
__global__ __launch_bounds__(256) void k_layout_rows(const int64_t* __restrict__ start, const int32_t* __restrict__ deg,
                                                      const int32_t* __restrict__ lay, int64_t P,
                                                      int2* __restrict__ rows) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P) return;
    rows[lay ? (int64_t)lay[q] : q] = make_int2((int)start[q], deg[q]);
}

// Point p's records at rows[p].x: each neighbour k's position and its own row (one thread
// per point; the model has been checked, so every index is in range).
__global__ __launch_bounds__(256) void k_build_nbr(const double* __restrict__ pos, int64_t P,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ idx, const int2* __restrict__ rows,
                                                    NbrRec* __restrict__ nbr, int32_t* __restrict__ nid) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t a = off[p], d = rows[p].x;
    const int n = rows[p].y;
    for (int j = 0; j < n; ++j) {
        const int32_t k = idx[a + j];
        NbrRec r;
        r.x = pos[3 * (int64_t)k];
        r.y = pos[3 * (int64_t)k + 1];
        r.z = pos[3 * (int64_t)k + 2];
        r.start = rows[k].x;
        r.deg = rows[k].y;
        nbr[d + j] = r;
        nid[d + j] = k;
    }
}

__global__ __launch_bounds__(256) void k_check_off(const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                                                    const double* __restrict__ pos, int64_t P, int64_t E,
                                                    int32_t* __restrict__ bad) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    int64_t a = off[p], b = off[p + 1];
    if (a > b || a < 0 || b > E || (p == 0 && a != 0) || (p == P - 1 && b != E)) {
        atomicOr(bad, 2);
        return;
    }
    for (int64_t e = a; e < b; ++e) {
        if (idx[e] < 0 || idx[e] >= P) atomicOr(bad, 1);
        if (idx[e] == p) atomicOr(bad, 4);
    }
    // |x| <= 1e150 keeps every squared distance of the walk finite
    for (int i = 0; i < 3; ++i)
        if (!(fabs(pos[3 * p + i]) <= 1e150)) atomicOr(bad, 8);
}

// Each row's records in ascending neighbour id, or in ascending key[id] when a key is
// given (insertion sort, one thread per row).  The walk's per-lane scan relies on it: a
// lane meets its candidates in ascending id (key), so keeping the first of equal
// distances keeps the smaller one.
__global__ __launch_bounds__(256) void k_sort_rows(const int2* __restrict__ rows, int64_t P,
                                                    NbrRec* __restrict__ nbr, int32_t* __restrict__ nid,
                                                    const int32_t* __restrict__ key) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t a = rows[p].x, b = a + rows[p].y;
    for (int64_t e = a + 1; e < b; ++e) {
        const NbrRec r = nbr[e];
        const int32_t k = nid[e];
        const int32_t kk = key ? key[k] : k;
        int64_t f = e - 1;
        while (f >= a && (key ? key[nid[f]] : nid[f]) > kk) {
            nbr[f + 1] = nbr[f];
            nid[f + 1] = nid[f];
            --f;
        }
        nbr[f + 1] = r;
        nid[f + 1] = k;
    }
}

// GL lanes (4, 8 or 16) walk one ray.  At every step lane s takes neighbours s,
// s+GL, ... of the current point's row (contiguous records sorted by id, so a
// group reads whole cache lines and a lane meets its candidates in ascending
// id; a lane's loads are issued four at a time) and keeps its best forward
// candidate (least D, the first of equal D) together with that candidate's own CSR row (start,
// degree, held in the record, so the next step's loads depend on nothing
// else).  The group then finds the lexicographic minimum of (D, id) in two
// DPP reductions (the minimum D, then the smallest id among the lanes that
// reach it; stages: mirror within the row for 16 lanes, mirror within the
// half-row for 8 or 16, then swap neighbours, then swap pairs), and every lane
// reads the winner's Z and row from the one lane that holds it with a ballot
// and ds_bpermute.  The result equals a sequential scan of the row.
//
// List entries are buffered across the group and written in blocks of RUNL =
// max(GL, 8) entries aligned to absolute list positions (ids 32 or 64 bytes, Z
// 64 or 128 bytes at addresses that are multiples of those sizes), so the lists
// reach memory as whole aligned segments.  Lane s holds entries s*EPL ..
// s*EPL + EPL - 1 of a block (EPL = RUNL / GL, one or two), in a ring of two
// blocks.  Every RUNL steps -- the same step for every group of the wave, so
// the stores are issued once per wave -- each group stores the last block it
// has completed (exactly one completes per RUNL steps); the first block of a
// list is masked below its start, and when the ray ends the group stores what
// is left (at most the two ring blocks).
enum TraceMode { TRACE_COUNT = 0, TRACE_WRITE = 1, TRACE_PADDED = 2 };


// Every source lane of these permutations lies in the reading lane's own group
// (groups of 4, 8 or 16 lanes move through the loop together), so no lane
// reads a disabled one and the bound-control value is never used.
template <int CTRL>
__device__ inline int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ inline double dpp_d(double v) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = dpp_i<CTRL>(p.x);
    p.y = dpp_i<CTRL>(p.y);
    return __builtin_bit_cast(double, p);
}

struct Cand {
    double D, Z;
    int32_t e, start, deg;  // e: record index (in a row sorted by id, the same order as the id)
};

template <int CTRL>
__device__ inline int dpp_min_i(int v) {
    const int o = dpp_i<CTRL>(v);
    return o < v ? o : v;
}

template <int CTRL>
__device__ inline double dpp_min_d(double v) {
    return __builtin_fmin(v, dpp_d<CTRL>(v));
}

__device__ inline int bperm_i(int src_lane, int v) { return __builtin_amdgcn_ds_bpermute(src_lane << 2, v); }

__device__ inline double bperm_d(int src_lane, double v) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = bperm_i(src_lane, p.x);
    p.y = bperm_i(src_lane, p.y);
    return __builtin_bit_cast(double, p);
}

constexpr int DPP_ROW_MIRROR = 0x140;   // lane i <-> 15-i within each 16 lanes
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7-i within each 8 lanes
constexpr int DPP_SWAP1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int DPP_SWAP2 = 0x4E;         // quad_perm [2,3,0,1]

// Minimum over the GL lanes of a group, left in every lane of it.
template <int GL>
__device__ inline double group_min_d(double v) {
    if (GL == 16) v = dpp_min_d<DPP_ROW_MIRROR>(v);
    if (GL >= 8) v = dpp_min_d<DPP_HALF_MIRROR>(v);
    v = dpp_min_d<DPP_SWAP1>(v);
    return dpp_min_d<DPP_SWAP2>(v);
}

template <int GL>
__device__ inline int group_min_i(int v) {
    if (GL == 16) v = dpp_min_i<DPP_ROW_MIRROR>(v);
    if (GL >= 8) v = dpp_min_i<DPP_HALF_MIRROR>(v);
    v = dpp_min_i<DPP_SWAP1>(v);
    return dpp_min_i<DPP_SWAP2>(v);
}

// Work order.  Without `order`, ray L is slot L (origin-major).  With `order`
// (a permutation of origin positions, spatially sorted) ray L is direction
// L / n_origins of origin order[L % n_origins]: concurrent waves walk nearby
// origins in the same direction and share most of the rows they read.  With
// `ray_order` (n_rays origin positions, from k_length_order) ray L is direction
// L / n_origins of origin ray_order[L]: the same windows of nearby origins,
// their rays taken in order of length.  Blocks are renumbered so that each XCD
// (own L2) takes runs of 16 consecutive blocks, the XCDs' runs side by side
// (xcd_block, XCD_RUN_WALK).
template <int MODE, int GL>
__global__ __launch_bounds__(TRACE_BLOCK, GL == 4 ? 4 : 1) void k_trace(const double* __restrict__ pos,
                                                        const int2* __restrict__ rows,
                                                        const NbrRec* __restrict__ nbr,
                                                        const int32_t* __restrict__ nid, int64_t P,
                                                        const int32_t* __restrict__ origins, int64_t n_origins,
                                                        int64_t R, const double* __restrict__ dirs, int per_origin,
                                                        int32_t* __restrict__ lens, const int64_t* __restrict__ ray_off,
                                                        int32_t* __restrict__ ids, double* __restrict__ Zout,
                                                        int64_t capacity, int32_t* __restrict__ err,
                                                        const int32_t* __restrict__ order,
                                                        const int32_t* __restrict__ ray_order, int n_xcd) {
    static_assert(GL == 4 || GL == 8 || GL == 16, "4, 8 or 16 lanes per ray");
    constexpr int U = 32 / GL;  // candidates per lane per pass: a whole row of up to 32 in one round of loads
    const int sub = threadIdx.x & (GL - 1);
    const int64_t two_r = 2 * R;
    const int64_t n_rays = n_origins * two_r;
    const int64_t nb = (n_rays * GL + blockDim.x - 1) / blockDim.x;  // logical blocks
    for (int64_t blk = xcd_block(blockIdx.x, gridDim.x, n_xcd, XCD_RUN_WALK); blk < nb; blk += gridDim.x) {
    const int64_t L = (blk * (int64_t)blockDim.x + threadIdx.x) / GL;
    if (L >= n_rays) continue;  // whole groups leave together
    int64_t oi, rr;
    if (ray_order) {
        rr = L / n_origins;
        oi = ray_order[L];
    } else if (order) {
        const int64_t dslot = L / n_origins;
        oi = order[L - dslot * n_origins];
        rr = dslot;
    } else {
        oi = L / two_r;
        rr = L - oi * two_r;
    }
    const int64_t ray = oi * two_r + rr;
    const int64_t r = rr >> 1;
    const int64_t o = origins ? (int64_t)origins[oi] : oi;
    if (o < 0 || o >= P) {  // invalid origin id: empty ray, error latched
        if (sub == 0) {
            if (MODE != TRACE_WRITE) lens[ray] = 0;
            if (MODE != TRACE_COUNT) atomicOr(err, ERRBIT_ORIGIN);
        }
        continue;
    }
    const double* dv = dirs + 3 * ((per_origin ? oi * R : 0) + r);
    double dx = dv[0], dy = dv[1], dz = dv[2];
    if (rr & 1) {
        dx = -dx;
        dy = -dy;
        dz = -dz;
    }
    const double ox = pos[3 * o], oy = pos[3 * o + 1], oz = pos[3 * o + 2];
    int64_t base = 0;
    int32_t room = 0;
    if (MODE == TRACE_WRITE) {
        base = ray_off[ray];
        int64_t rm = ray_off[ray + 1] - base;
        if (base + rm > capacity) rm = capacity - base;
        room = (int32_t)(rm < 0 ? 0 : rm);
    } else if (MODE == TRACE_PADDED) {
        base = ray * capacity;  // capacity = slots per ray
        room = (int32_t)capacity;
    }
    const int2 row0 = rows[o];
    int32_t e0 = row0.x, deg = row0.y;
    int32_t n = 0;
    double Zc = 0.0;
    constexpr int RUNL = GL >= 8 ? GL : 8;  // entries per stored block
    constexpr int EPL = RUNL / GL;          // entries per lane per block
    int32_t ke[2 * EPL];                    // the ring: [block][entry] as record indices
    double kz[2 * EPL];
#pragma unroll
    for (int i = 0; i < 2 * EPL; ++i) {
        ke[i] = 0;
        kz[i] = 0.0;
    }
    // end of the last stored block (blocks before the one holding `base` count as stored)
    int64_t p_last = (base & ~(int64_t)(RUNL - 1)) - 1;
    // the group's EPL entries of the block starting at S (ring half rb), positions below
    // `lo` and from `hi` on left out
    auto store_block = [&](int64_t S, int rb, int64_t lo, int64_t hi) {
        const int64_t q = S + sub * EPL;
        if (EPL == 2 && q >= lo && q + 1 < hi) {
            *(int2*)(ids + q) = make_int2(nid[ke[2 * rb]], nid[ke[2 * rb + 1]]);
            *(double2*)(Zout + q) = make_double2(kz[2 * rb], kz[2 * rb + 1]);
        } else {
#pragma unroll
            for (int e = 0; e < EPL; ++e)
                if (q + e >= lo && q + e < hi) {
                    ids[q + e] = nid[ke[rb * EPL + e]];
                    Zout[q + e] = kz[rb * EPL + e];
                }
        }
    };
    for (int32_t step = 0; step < (int32_t)P; ++step) {
        Cand b;
        b.D = __builtin_inf();
        b.Z = 0.0;
        b.e = INT32_MAX;
        b.start = 0;
        b.deg = 0;
        // GL lanes x U candidates per pass (32 entries); a lane's U loads are issued together
        for (int32_t i0 = 0; i0 < deg; i0 += U * GL) {
            NbrRec rec[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t i = i0 + u * GL + sub;
                if (i < deg) rec[u] = nbr[e0 + i];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t i = i0 + u * GL + sub;
                if (i >= deg) continue;
                const double Rx = rec[u].x - ox, Ry = rec[u].y - oy, Rz = rec[u].z - oz;
                const double Zk = __builtin_fma(Rz, dz, __builtin_fma(Ry, dy, Rx * dx));
                if (!(Zk > Zc)) continue;
                const double qx = __builtin_fma(-Zk, dx, Rx), qy = __builtin_fma(-Zk, dy, Ry),
                             qz = __builtin_fma(-Zk, dz, Rz);
                const double Dk = __builtin_fma(qz, qz, __builtin_fma(qy, qy, qx * qx));
                if (Dk < b.D) {  // ascending ids within the lane: the first of equal D has the smaller id
                    b.D = Dk;
                    b.Z = Zk;
                    b.e = (int32_t)(e0 + i);
                    b.start = rec[u].start;
                    b.deg = rec[u].deg;
                }
            }
        }
        // group minimum of (D, record index); within the sorted row the smaller
        // index is the smaller id, so this is the minimum of (D, id)
        const double Dmin = group_min_d<GL>(b.D);
        const int32_t emin = group_min_i<GL>(b.D == Dmin ? b.e : INT32_MAX);
        if (emin == INT32_MAX) break;  // no forward neighbour: the ray leaves the model
        // the winner's Z and row, read from the lane that holds it
        const uint64_t won = __ballot(b.D == Dmin && b.e == emin);
        const int gbase = (int)(threadIdx.x & 63) & ~(GL - 1);
        const uint32_t gbits = (uint32_t)(won >> gbase) & (uint32_t)((1ull << GL) - 1);
        const int src = gbase + __builtin_ctz(gbits);
        const double Zn = bperm_d(src, b.Z);
        const int32_t start_n = bperm_i(src, b.start);
        const int32_t deg_n = bperm_i(src, b.deg);
        if (MODE != TRACE_COUNT) {
            if (n >= room) {
                if (sub == 0) atomicOr(err, ERRBIT_CAPACITY);
                break;
            }
            const int64_t at = base + n;  // absolute list position of this entry
            const int o = (int)(at & (RUNL - 1));
            if (sub == o / EPL) {
                const int k = (int)((at / RUNL) & 1) * EPL + o % EPL;
#pragma unroll
                for (int i = 0; i < 2 * EPL; ++i)
                    if (i == k) {
                        ke[i] = emin;
                        kz[i] = Zn;
                    }
            }
            if ((n & (RUNL - 1)) == RUNL - 1) {  // the step of the wave's stores
                const int64_t Pend = at - ((at + 1) & (RUNL - 1));  // end of the last completed block
                const int64_t S = Pend - (RUNL - 1);
                store_block(S, (int)((S / RUNL) & 1), base, at + 1);
                p_last = Pend;
            }
        }
        ++n;
        e0 = start_n;
        deg = deg_n;
        Zc = Zn;
    }
    if (MODE != TRACE_COUNT) {  // what is left: at most the two ring blocks after p_last
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2) {
            const int64_t S = p_last + 1 + (int64_t)b2 * RUNL;
            if (S < base + n) store_block(S, (int)((S / RUNL) & 1), base, base + n);
        }
    }
    if (MODE != TRACE_WRITE && sub == 0) lens[ray] = n;
    // a ray shorter than its slot leaves entries unwritten: the offsets do not match this walk
    if (MODE == TRACE_WRITE && sub == 0 && n < room) atomicOr(err, ERRBIT_CAPACITY);
    }
}

// Padded slots (ray * cap) -> compacted lists at ray_off.  Eight lanes per ray.
__global__ __launch_bounds__(256) void k_compact(const int32_t* __restrict__ pids, const double* __restrict__ pZ,
                                                  int64_t cap, const int64_t* __restrict__ ray_off, int64_t n_rays,
                                                  int32_t* __restrict__ ids, double* __restrict__ Z) {
    const int sub = threadIdx.x & 7;
    const int64_t nb = (n_rays * 8 + blockDim.x - 1) / blockDim.x;
    for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
        const int64_t ray = (blk * (int64_t)blockDim.x + threadIdx.x) >> 3;
        if (ray >= n_rays) continue;
        const int64_t b = ray_off[ray], n = ray_off[ray + 1] - b;
        const int64_t src = ray * cap;
        for (int64_t j = sub; j < n && j < cap; j += 8) {
            ids[b + j] = pids[src + j];
            Z[b + j] = pZ[src + j];
        }
    }
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
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

inline int64_t blocks_for(int64_t n, int b) { return (n + b - 1) / b; }

}  // namespace

hipError_t launch_check_model(const rt_model* m, int32_t* bad, hipStream_t s) {
    hipLaunchKernelGGL(k_check_off, dim3((unsigned)blocks_for(m->P, 256)), dim3(256), 0, s, m->off, m->idx, m->pos, m->P,
                       m->E, bad);
    return hipGetLastError();
}

static size_t al256(size_t v) { return (v + 255) / 256 * 256; }

size_t build_nbr_workspace(int64_t P) {
    return al256(sizeof(int32_t) * (size_t)P) + al256(sizeof(int64_t) * (size_t)(P + 1)) + al256(scan_workspace(P));
}

hipError_t launch_build_nbr(const rt_model* m, const int32_t* key, const int32_t* lay, void* ws, hipStream_t s) {
    int32_t* deg = (int32_t*)ws;
    int64_t* start = (int64_t*)((char*)ws + al256(sizeof(int32_t) * (size_t)m->P));
    void* scan_ws = (char*)start + al256(sizeof(int64_t) * (size_t)(m->P + 1));
    const unsigned g = (unsigned)blocks_for(m->P, 256);
    hipLaunchKernelGGL(k_layout_deg, dim3(g), dim3(256), 0, s, m->off, lay, m->P, deg);
    hipError_t e = launch_scan(deg, m->P, start, scan_ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_layout_rows, dim3(g), dim3(256), 0, s, start, deg, lay, m->P, m->rows);
    if (m->E > 0) {
        hipLaunchKernelGGL(k_build_nbr, dim3(g), dim3(256), 0, s, m->pos, m->P, m->off, m->idx, m->rows, m->nbr, m->nid);
        hipLaunchKernelGGL(k_sort_rows, dim3(g), dim3(256), 0, s, m->rows, m->P, m->nbr, m->nid, key);
    }
    return hipGetLastError();
}

template <int MODE>
static hipError_t trace_launch(const rt_model* m, const int32_t* origins, int64_t n_origins, int64_t R,
                               const double* dirs, int per_origin, int32_t* lens, const int64_t* ray_off,
                               int32_t* ids, double* Z, int64_t capacity, const int32_t* order,
                               const int32_t* ray_order, int gl, hipStream_t s) {
    const int64_t n = n_origins * 2 * R;
    if (n == 0) return hipSuccess;
    if (gl != 8 && gl != 16) gl = 4;  // 0 and other values: the default, 4 lanes
    int32_t* ew = MODE == TRACE_COUNT ? nullptr : error_word();
    if (gl == 16)
        hipLaunchKernelGGL((k_trace<MODE, 16>), dim3(capped_blocks(blocks_for(n * 16, TRACE_BLOCK))), dim3(TRACE_BLOCK), 0, s, m->pos,
                           m->rows, m->nbr, m->nid, m->P, origins, n_origins, R, dirs, per_origin, lens, ray_off, ids, Z,
                           capacity, ew, order, ray_order, num_xcds());
    else if (gl == 8)
        hipLaunchKernelGGL((k_trace<MODE, 8>), dim3(capped_blocks(blocks_for(n * 8, TRACE_BLOCK))), dim3(TRACE_BLOCK), 0, s, m->pos,
                           m->rows, m->nbr, m->nid, m->P, origins, n_origins, R, dirs, per_origin, lens, ray_off, ids, Z,
                           capacity, ew, order, ray_order, num_xcds());
    else
        hipLaunchKernelGGL((k_trace<MODE, 4>), dim3(capped_blocks(blocks_for(n * 4, TRACE_BLOCK))), dim3(TRACE_BLOCK), 0, s, m->pos,
                           m->rows, m->nbr, m->nid, m->P, origins, n_origins, R, dirs, per_origin, lens, ray_off, ids, Z,
                           capacity, ew, order, ray_order, num_xcds());
    return hipGetLastError();
}

hipError_t launch_trace_count(const rt_model* m, const int32_t* origins, int64_t n_origins, int64_t R,
                              const double* dirs, int per_origin, int32_t* lens, hipStream_t s,
                              const int32_t* order, int gl) {
    return trace_launch<TRACE_COUNT>(m, origins, n_origins, R, dirs, per_origin, lens, nullptr, nullptr, nullptr, 0,
                                     order, nullptr, gl, s);
}

hipError_t launch_trace_write(const rt_model* m, const int32_t* origins, int64_t n_origins, int64_t R,
                              const double* dirs, int per_origin, const int64_t* ray_off, int32_t* ids,
                              double* Z, int64_t capacity, hipStream_t s, const int32_t* order, int gl,
                              const int32_t* ray_order) {
    return trace_launch<TRACE_WRITE>(m, origins, n_origins, R, dirs, per_origin, nullptr, ray_off, ids, Z, capacity,
                                     order, ray_order, gl, s);
}

hipError_t launch_trace_padded(const rt_model* m, const int32_t* origins, int64_t n_origins, int64_t R,
                               const double* dirs, int per_origin, int32_t* lens, int32_t* pids, double* pZ,
                               int64_t cap, hipStream_t s, const int32_t* order, int gl) {
    return trace_launch<TRACE_PADDED>(m, origins, n_origins, R, dirs, per_origin, lens, nullptr, pids, pZ, cap, order,
                                      nullptr, gl, s);
}

// For every direction slot d, the windows of LEN_WINDOW consecutive positions
// of `order` re-sorted by the length of their ray d (ties keep the given order;
// a bitonic sort of 32-bit keys (length << 8 | position in window) in LDS).
// out[d * n_o + k] is an origin position.  Rays walked by one wave then end at
// nearly the same step instead of the wave running until its longest ray ends,
// while each window stays a compact group of nearby origins.
constexpr int LEN_WINDOW = 64;

__global__ __launch_bounds__(LEN_WINDOW) void k_length_order(const int32_t* __restrict__ lens,
                                                             const int32_t* __restrict__ order, int64_t n_o,
                                                             int64_t two_r, int32_t* __restrict__ out) {
    __shared__ uint32_t sk[LEN_WINDOW];
    __shared__ int32_t so[LEN_WINDOW];
    const int t = threadIdx.x;
    const int64_t n_win = (n_o + LEN_WINDOW - 1) / LEN_WINDOW;
    for (int64_t w = blockIdx.x; w < n_win * two_r; w += gridDim.x) {
        const int64_t d = w / n_win;
        const int64_t k = (w - d * n_win) * LEN_WINDOW + t;
        uint32_t key = 0xFFFFFFFFu;  // past the end: sorts last
        int32_t oi = 0;
        if (k < n_o) {
            oi = order[k];
            const int32_t len = lens[(int64_t)oi * two_r + d];
            const uint32_t lc = len <= 0 ? 0u : (len >= 0xFFFFFE ? 0xFFFFFEu : (uint32_t)len);
            key = (lc << 8) | (uint32_t)t;
        }
        sk[t] = key;
        so[t] = oi;
        __syncthreads();
        for (int size = 2; size <= LEN_WINDOW; size <<= 1)
            for (int j = size >> 1; j > 0; j >>= 1) {
                const int u = t ^ j;
                if (u > t) {
                    const uint32_t a = sk[t], b = sk[u];
                    if ((a > b) == ((t & size) == 0)) {
                        sk[t] = b;
                        sk[u] = a;
                        const int32_t x = so[t];
                        so[t] = so[u];
                        so[u] = x;
                    }
                }
                __syncthreads();
            }
        if (k < n_o) out[d * n_o + k] = so[t];
        __syncthreads();  // the next window reuses the tables
    }
}

hipError_t launch_length_order(const int32_t* lens, const int32_t* order, int64_t n_origins, int64_t R,
                               int32_t* out, hipStream_t s) {
    const int64_t n_win = (n_origins + LEN_WINDOW - 1) / LEN_WINDOW;
    if (n_win == 0 || R == 0) return hipSuccess;
    hipLaunchKernelGGL(k_length_order, dim3(capped_blocks(n_win * 2 * R)), dim3(LEN_WINDOW), 0, s, lens, order,
                       n_origins, 2 * R, out);
    return hipGetLastError();
}

hipError_t launch_compact(const int32_t* pids, const double* pZ, int64_t cap, const int64_t* ray_off, int64_t n_rays,
                          int32_t* ids, double* Z, hipStream_t s) {
    if (n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3(capped_blocks(blocks_for(n_rays * 8, 256))), dim3(256), 0, s, pids, pZ, cap, ray_off, n_rays,
                       ids, Z);
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
    hipLaunchKernelGGL(k_fill_i32, dim3(capped_blocks(blocks_for(n, 256))), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace rt
