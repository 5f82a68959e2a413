// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rt.h"

namespace rt {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
rt_status fail(rt_status code, const std::string& msg);
rt_status hip_fail(hipError_t e, const char* what);
#define RT_HIP(call)                                             \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return ::rt::hip_fail(e_, #call);  \
    } while (0)

// Device-side error word (per device), written by kernels with atomicOr.
enum : int32_t { ERRBIT_CAPACITY = 1, ERRBIT_NONFINITE = 2, ERRBIT_ORIGIN = 4, ERRBIT_STEP = 8 };
int32_t* error_word();  // device address for the current device, nullptr on failure
int num_cus();
int num_xcds();

// A dispatch covers at most 2^32 - 1 work-items per dimension; kernels whose
// logical index space can be larger loop over it in rounds of at most
// MAX_GRID_BLOCKS workgroups.
constexpr int64_t MAX_GRID_BLOCKS = (int64_t)1 << 22;
inline unsigned capped_blocks(int64_t n_blocks) {
    return (unsigned)(n_blocks < 1 ? 1 : (n_blocks > MAX_GRID_BLOCKS ? MAX_GRID_BLOCKS : n_blocks));
}

// Workgroups are dispatched to the XCDs round-robin (workgroup b runs on XCD
// b mod n).  This renumbering gives each XCD runs of R consecutive logical
// blocks, the runs of the n XCDs side by side: logical blocks [k n R, (k+1) n R)
// are run k of every XCD (XCD x takes [k n R + x R, k n R + (x+1) R)).  Work
// adjacent in the logical order then shares an L2 within a run, while all XCDs
// work on one stretch of the logical order at a time, so what they read
// together also stays small in the Infinity Cache that they share (one
// contiguous range per XCD made the walk of the 64-cloud batch 14% slower).  A
// bijection of [0, G) for any grid size G: the blocks past the last whole
// group of n runs keep their own number.  Run lengths: the walk 16 workgroups
// (16 windows of 64 origins), the sweep 256 (1024 items); measured on the batch
// and the octree.
constexpr int64_t XCD_RUN_WALK = 16;
constexpr int64_t XCD_RUN_SWEEP = 256;
__device__ inline int64_t xcd_block(int64_t b, int64_t G, int n, int64_t R) {
    if (n <= 1) return b;
    const int64_t span = (int64_t)n * R, full = G / span * span;
    if (b >= full) return b;
    const int64_t x = b % n, i = b / n;
    return (i / R) * span + x * R + (i % R);
}

// ---------------------------------------------------------------- HEALPix (host)
// Centre of ring-scheme pixel p at resolution nside (unit vector) and its ring.
void hp_centre(int64_t nside, int64_t p, double v[3], int64_t* ring);
// Antipodal pixel (exact integer map: opposite ring, half a turn along it).
int64_t hp_antipode(int64_t nside, int64_t p);

// ---------------------------------------------------------------- handles
struct DevTables {
    int device = -1;
    double* dirs = nullptr;  // [n][R][3]
    double* w2 = nullptr;    // [n][R]
};

}  // namespace rt

struct rt_dirset {
    int32_t lmin = 0, lmax = 0;
    int64_t R = 0;          // pairs per origin
    int64_t n_origins = 0;  // 0: shared set
    // shared sets: host tables
    std::vector<int64_t> pix;
    std::vector<int32_t> level;
    std::vector<double> dirs, w2;
    // device tables (uploaded lazily for shared sets, owned for adaptive sets)
    rt::DevTables dev;
    int64_t* dev_pix = nullptr;   // adaptive only
    int32_t* dev_level = nullptr; // adaptive only
    rt_status ensure_device();
    const double* d_dirs() const { return dev.dirs; }
    const double* d_w2() const { return dev.w2; }
};

// One neighbour entry as the tracer reads it (32 bytes, two 16-byte loads): the
// neighbour's position and its own CSR row (start, degree), so a step needs no
// further load to continue from the chosen neighbour.  Rows are sorted by
// neighbour id; the ids themselves sit in a separate array in the same order.
struct alignas(16) NbrRec {
    double x, y, z;
    int32_t start;
    int32_t deg;
};

struct rt_model {
    const double* pos = nullptr;
    int64_t P = 0;
    const int64_t* off = nullptr;
    const int32_t* idx = nullptr;
    int64_t E = 0;
    const float* vel = nullptr;
    NbrRec* nbr = nullptr;  // owned: neighbour records, rows in Morton order of the points, each sorted by id
    int32_t* nid = nullptr; // owned: the neighbour id of each record
    int2* rows = nullptr;   // owned: per point {row start, degree}
    int device = -1;
    // host copy of the positions, made on first need (spatial orders of plans); the
    // positions may not change while the handle lives
    mutable std::vector<double> host_pos;
    mutable std::mutex host_mu;
};

namespace rt {

// ---------------------------------------------------------------- kernels (launchers)
// trace.hip
// Checks of a model's CSR and positions (bits of *bad: 1 index out of range, 2 bad offsets,
// 4 self neighbour, 8 position not finite or beyond 1e150).
hipError_t launch_check_model(const rt_model* m, int32_t* bad, hipStream_t s);
// Records, ids and rows of a checked model: the rows laid out in the point order `lay`
// (device [P], NULL: point order), each row in ascending key[id] (key NULL: ascending id);
// ws: build_nbr_workspace(P) bytes.
size_t build_nbr_workspace(int64_t P);
hipError_t launch_build_nbr(const rt_model* m, const int32_t* key, const int32_t* lay, void* ws, hipStream_t s);
// `order` (optional): spatially sorted permutation of origin positions; the
// rays are then walked direction-major in that origin order.  gl: lanes per
// ray, 4, 8 or 16 (anything else: 4).  `ray_order` (optional, n_rays origin
// positions from launch_length_order): the write walk takes the rays of each
// direction in that order instead.
hipError_t launch_trace_count(const rt_model* m, const int32_t* origins, int64_t n_origins, int64_t R,
                              const double* dirs, int per_origin, int32_t* lens, hipStream_t s,
                              const int32_t* order = nullptr, int gl = 0);
hipError_t launch_trace_write(const rt_model* m, const int32_t* origins, int64_t n_origins, int64_t R,
                              const double* dirs, int per_origin, const int64_t* ray_off, int32_t* ids,
                              double* Z, int64_t capacity, hipStream_t s, const int32_t* order = nullptr,
                              int gl = 0, const int32_t* ray_order = nullptr);
hipError_t launch_trace_padded(const rt_model* m, const int32_t* origins, int64_t n_origins, int64_t R,
                               const double* dirs, int per_origin, int32_t* lens, int32_t* pids, double* pZ,
                               int64_t cap, hipStream_t s, const int32_t* order = nullptr, int gl = 0);
// Per direction, windows of 64 consecutive positions of `order` (n_origins
// origin positions) re-sorted by the length of their ray (lens in slot order
// o * 2R + slot, from a count pass), ties in the given order: out[d * n_origins
// + k], n_origins * 2R entries, for launch_trace_write's ray_order.
hipError_t launch_length_order(const int32_t* lens, const int32_t* order, int64_t n_origins, int64_t R,
                               int32_t* out, hipStream_t s);
hipError_t launch_compact(const int32_t* pids, const double* pZ, int64_t cap, const int64_t* ray_off, int64_t n_rays,
                          int32_t* ids, double* Z, hipStream_t s);
size_t scan_workspace(int64_t n);
hipError_t launch_scan(const int32_t* lens, int64_t n, int64_t* off, void* ws, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

// solve.hip
struct SolveLaunch {
    const int32_t* origins;
    int64_t n_origins;
    int64_t R;
    const double* dirs;
    const double* w2;
    int per_origin;
    const int64_t* ray_off;
    const int32_t* ray_ids;
    const double* ray_Z;
    const void* chi;
    const void* eta;
    int64_t ld;
    int32_t F;
    int32_t n_blocks;
    int32_t blk_start[RT_MAX_FREQ_BLOCKS + 1];
    double inv_dx[RT_MAX_FREQ_BLOCKS];
    double dx[RT_MAX_FREQ_BLOCKS];
    const float* vel;
    const double* I_bc;
    void* u;
    void* J;
    double dtau_max_rcp;   // 1/dtau_max (adaptive optical-depth increments), 0 = off
    double dv_max_rcp;     // 1/dv_max (adaptive velocity sampling), 0 = off
    int32_t max_sub;       // cap on the sub-steps of one interval
    // scheduling
    int32_t schedule;
    const int32_t* items;  // binned order, or nullptr
    const int32_t* order;  // spatial order of origin positions (direct launch, direction-major), or nullptr
    const int32_t* pair_order;  // with order: the sweep's own order per pair ([R][n_origins]), or nullptr
    int32_t* queue;        // persistent counter, or nullptr
    int32_t grid_waves;    // persistent grid size in waves
    int32_t n_bins;
    int32_t bins_per_octave;  // bin of a line of N points: floor(bins_per_octave * log2 N)
    int32_t* bin_counts;   // [n_bins+1] scratch
    int32_t* bin_cursor;   // [n_bins] scratch
    int32_t* err;          // device error word
    int64_t P;             // number of points (origin ids are checked against it)
    int n_xcd;             // XCDs for the block renumbering of the direct launch
    int group;             // sweep load-group size (4 or 8)
    int small_tables;      // chi and eta each below 4 GiB: 32-bit row offsets in the sweep
    int scheme;            // RT_SCHEME_FEAUTRIER2 or RT_SCHEME_HERMITE
};
int64_t solve_items(const SolveLaunch& a);
// Items a persistent wave takes per queue atomic, the cap on its grid (waves per
// CU), and so the largest item count whose int32 queue counter cannot overflow.
constexpr int PERSIST_CHUNK = 16;
constexpr int MAX_WAVES_PER_CU = 256;
constexpr int64_t MAX_SOLVE_ITEMS = (int64_t)INT32_MAX - ((int64_t)1 << 26);
size_t bin_workspace(int64_t n_items, int32_t n_bins);
hipError_t launch_bin(const SolveLaunch& a, void* ws, int32_t** items_out, hipStream_t s);
hipError_t launch_solve(const SolveLaunch& a, int precision, hipStream_t s);
hipError_t launch_reduce(const SolveLaunch& a, int precision, hipStream_t s);

// api.hip: pieces of the solve and plan set-up shared by the whole-path entry points
rt_solve_opts default_solve_opts();
int32_t opts_bins(const rt_solve_opts& o);
int32_t opts_bins_per_octave(const rt_solve_opts& o);
// Validate the solve arguments and fill a launch description (lists may be set later).
rt_status fill_solve_launch(const rt_model* m, rt_dirset* set, const int32_t* origins, int64_t n_origins,
                            const int64_t* ray_off, const int32_t* ray_ids, const double* ray_Z, const void* chi,
                            const void* eta, int32_t dtype, int64_t ld, const rt_freq_grid* grid,
                            const double* I_bc, void* J, const rt_solve_opts& o, SolveLaunch& a);
// Morton order of the positions of the listed origins (host order of list positions).  With
// segments (n_seg > 0, seg[0..n_seg] ascending list positions) each segment is ordered on its own
// bounding box and the segments follow one another.  Synchronises `s` once (host copies).
hipError_t morton_order(const rt_model* m, const int32_t* origins, int64_t n_o, hipStream_t s,
                        std::vector<int32_t>& order, const int64_t* seg = nullptr, int n_seg = 0);
// Per-pair sweep orders (order.hip): for each pair r, the origin positions sorted by
// (segment, 2D Morton code across d_r, position along d_r).  A segment covers the origin
// positions below `end` not in an earlier one, inside the sphere (c, rho).
struct OrderSeg {
    int64_t end;
    double c[3];
    double rho;
};
size_t pair_order_workspace(int64_t n_o);
// pos, origins, segs (n_seg <= 65535) and out ([R][n_o]) on the device; dirs_host [R][3] on
// the host; ws: pair_order_workspace(n_o) bytes.  Asynchronous on s.
hipError_t build_pair_orders(const double* pos, int64_t P, const int32_t* origins, int64_t n_o, const double* dirs_host,
                             int64_t R, const OrderSeg* segs, int n_seg, int32_t* out, void* ws, hipStream_t s);

// The same order from host arrays: positions [P][3], origin ids (NULL: 0..n_o-1).
void morton_order_host(const double* pos, int64_t P, const int32_t* origins, int64_t n_o, std::vector<int32_t>& order,
                       const int64_t* seg, int n_seg);
// rt_model_create with the rows of the neighbour records in ascending key[id] (device [P],
// NULL: ascending id); the walk breaks ties of equal distance by that order.
// morton_rows: lay the rows of the records out in the Morton order of the points (else in
// point order, for points that are already so ordered).
rt_status model_create(const double* pos, int64_t P, const int64_t* nbr_off, const int32_t* nbr_idx, int64_t E,
                       const float* vel, const int32_t* key, bool morton_rows, hipStream_t s, rt_model** out);
// Plans: create with a given origin order (nullptr = Morton order of the origins), enqueue the
// whole step on a stream (what the plan's graph holds), and a counter that changes whenever the
// plan's graph is re-captured.
rt_status plan_create_ordered(const rt_model* m, rt_dirset* set, const int32_t* origins, int64_t n_origins,
                              const void* chi, const void* eta, int32_t dtype, int64_t ld, const rt_freq_grid* grid,
                              const double* I_bc, void* J, const rt_solve_opts* opts, hipStream_t s,
                              const std::vector<int32_t>* order, rt_plan** out,
                              const std::vector<OrderSeg>* segs = nullptr);
hipError_t plan_enqueue_step(rt_plan* p, hipStream_t s);
int64_t plan_version(const rt_plan* p);

// compute.hip: the chunked whole path (rt_compute_J) with its workspace carved by the caller
size_t compute_ws_fixed(int64_t n_origins, int64_t R, int64_t F, const rt_solve_opts& o);

}  // namespace rt
