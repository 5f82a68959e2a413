/*
 * rt.h -- C ABI of the MI355X (gfx950) ray-tracing radiative-transfer library.
 *
 * Given a point cloud with nearest-neighbour lists (Section 2.2: a point cloud
 * plus nearest-neighbour information is all the method needs), per-point
 * opacity chi(nu) and emissivity eta(nu) (Section 2.1: the ray tracer gathers
 * emissivities and opacities along each ray), per-point velocities
 * (Section 2.1.1) and a hierarchical HEALPix direction set (Section 2.1.3),
 * the library returns the mean intensity J[point][nu], the directional
 * integral of eq. 3 with the weights of eq. 4.
 *
 * Conventions for every entry point:
 *  - Every function returns rt_status: RT_OK (0) or a negative error code.
 *    rt_last_error() then holds a message (thread-local).  No C++ exception
 *    crosses this boundary.
 *  - "device" pointers are HIP device memory (e.g. torch tensors on cuda:0);
 *    "host" pointers are ordinary memory.  Buffers passed in are borrowed:
 *    the caller owns them and keeps them alive while a call or a handle that
 *    refers to them is in use.  Handles own only the small tables they build.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls marked
 *    "async" only enqueue work on it; errors found by the kernels afterwards
 *    are reported by rt_sync_status().
 *  - Layouts: pos float64 [P][3]; nbr_off int64 [P+1] (CSR, off[0] = 0);
 *    nbr_idx int32 [E]; vel float32 [P][3] in Doppler widths or NULL (static);
 *    chi, eta [P][ld] row-major, frequency contiguous, dtype RT_F32 or RT_F64;
 *    J [n_origins][F] of the same dtype.
 *  - Ray slots: ray s = o*2R + 2r (+n_r) or o*2R + 2r + 1 (-n_r) for origin
 *    position o in the origin list and pair r of R; ray_off[s] .. ray_off[s+1]
 *    delimits ray s in ray_ids / ray_Z.
 */
#ifndef RT_H
#define RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rt_status;
enum {
    RT_OK = 0,
    RT_ERR_ARG = -1,         /* bad argument, size or NULL pointer */
    RT_ERR_MESH = -2,        /* neighbour list out of range, self, duplicate or asymmetric */
    RT_ERR_OPACITY = -3,     /* chi <= 0 or non-finite */
    RT_ERR_CAPACITY = -4,    /* workspace or list capacity too small */
    RT_ERR_HIP = -5,         /* a HIP runtime call failed */
    RT_ERR_UNSUPPORTED = -6, /* nside not a power of two, level > 13, too many blocks */
    RT_ERR_NONFINITE = -7,   /* the solve produced a non-finite u */
    RT_ERR_STATE = -8,       /* handle used in the wrong state */
    RT_ERR_STEP = -9         /* RT_SCHEME_HERMITE: an optical-depth step beyond the rows' limit */
};

enum { RT_F32 = 1, RT_F64 = 2 };

#define RT_MAX_FREQ_BLOCKS 8
#define RT_MAX_LEVEL 13

/* Message of the last failing call on this thread ("" if none). */
const char* rt_last_error(void);
rt_status rt_version(int32_t* major, int32_t* minor);
/* sizeof(rt_solve_opts) and sizeof(rt_freq_grid) as the library was built, for
 * bindings that mirror the structs. */
rt_status rt_struct_sizes(size_t* solve_opts, size_t* freq_grid);

/* ------------------------------------------------------------------ direction sets
 * HEALPix ring-scheme pixels at level l (nside = 2^l) have equal area, 12*4^l of
 * them (Section 2.1.3).  Rays come in antipodal pairs (Section 2.1.3); the pair
 * member with the smaller ring index is canonical, its centre is the pair's
 * direction n_r, the partner ray is exactly -n_r.  A pair at level l carries
 * weight 2w, w = 1/(12*4^l) (eq. 4).  Sets are built on the host; the handle
 * uploads its tables to the current device on first use. */
typedef struct rt_dirset rt_dirset;

/* Every pair at level log2(nside), ascending canonical ring index (6*nside^2 pairs).
 * nside must be a power of two <= 2^RT_MAX_LEVEL. */
rt_status rt_dirset_uniform(int32_t nside, rt_dirset** out);

/* Adaptive per-origin sets (Section 2.1.3, Fig. 1): for each origin, the
 * directions to the sample points (sample_ids, host, n_sample ids) are
 * histogrammed at level lmax; pair counts are downgraded through the nested
 * hierarchy; starting from every pair at lmin, the top half of the active
 * pairs of each level (by count, ties to the smaller ring index) is refined.
 * The same number of pairs results for every origin: 6*4^lmin*((2^K-1)/2 + 2^K),
 * K = lmax-lmin (552 rays for lmin=1, lmax=4).  Built on the GPU (async on
 * `stream`); model positions and origins are device pointers. */
typedef struct rt_model rt_model;
rt_status rt_dirset_adaptive(const rt_model* model, int32_t lmin, int32_t lmax,
                             const int32_t* sample_ids_dev, int64_t n_sample,
                             const int32_t* origins_dev, int64_t n_origins,
                             void* stream, rt_dirset** out);

/* Pairs per origin, number of origins the set is specific to (0 = shared by all
 * origins), and levels. */
rt_status rt_dirset_info(const rt_dirset* set, int64_t* pairs, int64_t* n_origins,
                         int32_t* lmin, int32_t* lmax);

/* Copy the set to host: pix [n][R] canonical pixel ids at their level,
 * level [n][R], dirs [n][R][3], w2 [n][R], n = max(1, n_origins).  Any output
 * pointer may be NULL.  For adaptive sets this synchronises `stream`. */
rt_status rt_dirset_export(const rt_dirset* set, int64_t* pix, int32_t* level, double* dirs,
                           double* w2, void* stream);
rt_status rt_dirset_destroy(rt_dirset* set);

/* ------------------------------------------------------------------ model
 * Borrows the caller's device arrays for the handle's lifetime.  Validates the
 * neighbour lists on the device (indices in range, no self entries; error
 * RT_ERR_MESH) and the positions (finite, every coordinate of magnitude at most
 * 1e150 so that the walk's squared distances stay finite; error RT_ERR_ARG)
 * and synchronises on `stream` to read the verdict before anything is built.
 * Then builds a neighbour-record table (36 bytes per neighbour entry: position,
 * id, the neighbour's own row; each row sorted by id) that the tracer reads
 * instead of chasing nbr_idx into pos and nbr_off, with the rows laid out in
 * the Morton order of the points (computed on the host from a copy of the
 * positions, which the handle keeps for the spatial orders of plans; 24 bytes
 * of host memory per point).  The order of a point's neighbours in nbr_idx and
 * the order of the points do not affect any result.  The positions and lists
 * must not change while the handle lives. */
rt_status rt_model_create(const double* pos, int64_t P, const int64_t* nbr_off, const int32_t* nbr_idx,
                          int64_t E, const float* vel, void* stream, rt_model** out);
rt_status rt_model_destroy(rt_model* model);

/* Host-side checks of a model (for callers holding host copies, and tests):
 * offsets monotone from 0 to E, indices in range, no self or duplicate entries,
 * symmetric lists, finite positions, chi finite and > 0 over [P][F] with row
 * stride ld (chi may be NULL).  Returns the first error found. */
rt_status rt_validate_host(const double* pos, int64_t P, const int64_t* nbr_off, const int32_t* nbr_idx,
                           int64_t E, const void* chi, int32_t dtype, int64_t F, int64_t ld);

/* ------------------------------------------------------------------ tracing
 * Every ray of every listed origin walks the neighbour graph (Section 2.1,
 * Fig. 2): from the current point it steps to the forward neighbour closest to
 * the ray axis.  With R = x_k - x_origin (per axis, FP64) and d the ray
 * direction, in FP64 with the fused multiply-adds written out:
 *   Z_k = fma(R.z, d.z, fma(R.y, d.y, R.x d.x))      (projection)
 *   forward:  Z_k > Z_current (strict)
 *   q = fma(-Z_k, d, R) per axis,
 *   D_k = fma(q.z, q.z, fma(q.y, q.y, q.x q.x))      (squared distance to the axis)
 * the least D_k wins, equal D_k go to the smaller point id; the ray records
 * (k, Z_k) and continues from k; it ends where no neighbour is forward.  The
 * origin itself is not recorded.  Nothing else is contracted, so lists are
 * bit-exact and independent of launch shape.
 *
 * origins: device int32 [n_origins], or NULL for 0..n_origins-1. */

/* Ray lengths and offsets: ray_off (device int64 [n_origins*2R + 1]) receives
 * the exclusive scan of the lengths, ray_off[n_rays] the total.  Async.
 * ws: device scratch of at least rt_trace_count_workspace() bytes. */
rt_status rt_trace_count_workspace(const rt_dirset* set, int64_t n_origins, size_t* bytes);
rt_status rt_trace_count(const rt_model* model, const rt_dirset* set, const int32_t* origins,
                         int64_t n_origins, int64_t* ray_off, void* ws, size_t ws_bytes, void* stream);

/* Writes ray_ids (int32) and ray_Z (float64) of every ray at the offsets from
 * rt_trace_count; `capacity` is the length of both arrays.  A ray that would
 * write past its slot or past capacity is truncated, and a ray shorter than its
 * slot leaves the rest unwritten; both latch RT_ERR_CAPACITY for
 * rt_sync_status().  Async. */
rt_status rt_trace_write(const rt_model* model, const rt_dirset* set, const int32_t* origins,
                         int64_t n_origins, const int64_t* ray_off, int32_t* ray_ids, double* ray_Z,
                         int64_t capacity, void* stream);

/* Count, scan and write in one call: ray_off (device int64 [n_rays + 1]) gets
 * the offsets, ray_ids / ray_Z (device, `capacity` entries each) the lists, and
 * total_dev (device int64 [1]) the total number of entries -- written even when
 * it exceeds `capacity`, in which case the rays past it are truncated and
 * RT_ERR_CAPACITY is latched for rt_sync_status() (call again with a larger
 * capacity: the lists are deterministic).  ws: rt_trace_count_workspace()
 * bytes.  Async; allocates nothing. */
rt_status rt_trace(const rt_model* model, const rt_dirset* set, const int32_t* origins, int64_t n_origins,
                   int64_t* ray_off, int32_t* ray_ids, double* ray_Z, int64_t capacity, int64_t* total_dev,
                   void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ solve
 * Frequency grid: n_blocks blocks, block b holding len[b] consecutive
 * frequencies uniformly spaced by dx[b] Doppler widths (host arrays).
 * F = sum(len) <= ld.
 *
 * For every origin o and pair r, the line reverse(ray -n_r), o, ray +n_r is
 * assembled with coordinates s = (-Z reversed, 0, Z).  Optics are taken in the
 * frame of o along +n_r (Section 2.1.1): point q is shifted by
 * delta_q = n_r.(v_q - v_o)/dx_b frequency steps, chi'_q[f] is the linear
 * interpolation of chi_q at index f - delta_q within the block (indices clamped
 * to the block), eta' likewise, S = eta'/chi'.  dtau_d = (chi'_d + chi'_{d+1})/2 * ds_d.
 * The second-order Feautrier equation (eq. 1) with second-order boundary
 * conditions and incoming intensity I_bc[f] at both ends of every line is
 * eliminated from both ends towards o in rescaled form; u at o is kept.
 * J[o][f] = sum_r w2_r u_r[f], summed in ascending r (eq. 3, eq. 4).
 *
 * precision RT_F64: all FP64 (tables must be RT_F64).  RT_F32: tables RT_F32,
 * sweep in FP32; ds is always formed in FP64 from the FP64 Z.  The rows are
 * carried per unit inner step (F = dtau G, Z = dtau Y), so the only
 * elimination coefficient, (dtau_{d-1} + dtau_d)/2, is in FP32 exactly its FP64
 * value rounded once: every row, however small its steps, has FP64
 * coefficients, and no row needs a separate FP64 path (so there is no
 * threshold option for one). */
typedef struct {
    int32_t n_blocks;
    const int32_t* len; /* host [n_blocks] */
    const double* dx;   /* host [n_blocks] */
    const double* x0;   /* host [n_blocks]: frequency of the block's first point in Doppler widths
                           about the line centre, x = x0[b] + j dx[b]; NULL = each block centred,
                           x0 = -(len-1) dx / 2.  Only the closure's features read it. */
} rt_freq_grid;

enum { RT_SCHED_DIRECT = 0, RT_SCHED_BINNED = 1, RT_SCHED_SPATIAL = 2 };

typedef struct {
    int32_t precision;        /* RT_F32 or RT_F64 */
    int32_t schedule;         /* RT_SCHED_DIRECT: one wave per (origin, pair, 64-frequency chunk) in
                                 slot order; RT_SCHED_BINNED: persistent waves draining a length-binned
                                 queue, longest lines first, 16 items per queue atomic (plans: the
                                 origins' Morton order inside each bin); RT_SCHED_SPATIAL (plans only): sweep items
                                 direction by direction, each XCD taking runs of 256 consecutive
                                 workgroups (the XCDs' runs side by side), with a uniform
                                 set each pair's items in that pair's line order (origins sorted by the
                                 2D Morton code of their position across the pair's direction, then
                                 along it; built on the device when the plan is configured, R x
                                 n_origins int32 of device memory, skipped above 2 GiB) and otherwise in
                                 the Morton order of the origins' positions -- concurrent waves then
                                 read mostly the same rows and the L2s hold them.  A plan's walk always
                                 uses the Morton order. */
    int32_t waves_per_cu;     /* persistent grid size in waves per CU (0 = 32; at most 256) */
    int32_t n_bins;           /* length bins for RT_SCHED_BINNED (0 = default 64, at most 128) */
    int32_t bins_per_octave;  /* RT_SCHED_BINNED bin edges: a pair whose line holds N points goes to bin
                                 floor(bins_per_octave * log2 N) (the last bin open-ended); 1, 2, 4 or
                                 8 (0 = 4, quarter octaves) */
    int32_t group;            /* sweep: line points whose loads are issued together, 4 or 8 (0 = 4) */
    int32_t trace_lanes;      /* plans: lanes walking one ray, 4, 8 or 16 (0 = 4) */
    int64_t padded_trace_budget; /* plans, RT_WALK_PADDED: bytes allowed for single-pass tracing into
                                    padded per-ray slots (longest ray x 12 bytes per ray); 0 = 32 GiB;
                                    beyond it, or < 0, the walk takes two passes (count, then write) */
    int32_t walk;             /* plans: RT_WALK_EXACT (0): every run walks each ray once straight into
                                 its slot of the lists sized by the count pass at creation (each
                                 direction's rays taken in windows of 64 nearby origins sorted by the
                                 lengths that pass found, so the rays of a wave end together; 4 bytes
                                 per ray of device memory); a ray whose length then differs from its
                                 slot latches RT_ERR_CAPACITY.
                                 RT_WALK_PADDED: once into padded slots, then scan and compaction.
                                 RT_WALK_TWO_PASS: count, scan, write on every run. */
    double dtau_max;          /* > 0: adaptive optical-depth increments (Section 2.1.2, eq. 2): the
                                 interval between line points d, d+1 is split into
                                 n = ceil(max(chi'_d, chi'_{d+1}) ds_d / dtau_max) equal parts
                                 (chi' Doppler-shifted, evaluated in FP64 as (1-t) chi_a + t chi_b;
                                 the product times the reciprocal of dtau_max rounded once), chi'
                                 and eta' interpolated linearly between the end points; 0 = off */
    int32_t max_substeps;     /* cap on n (and on m below) per interval (0 = 1024) */
    double dv_max;            /* > 0 (moving media): adaptive velocity sampling (Section 2.1.1), before
                                 the optical-depth split: with p_d = n_r.(v_d - v_o) the interval d, d+1
                                 gets m = ceil(|p_{d+1} - p_d| / dv_max) equal parts (Doppler widths;
                                 the reciprocal rounded once); a point at weight w = j/m from the point
                                 of smaller line coordinate carries p = (1-w) p_d + w p_{d+1} and the
                                 optics (1-w) X_d + w X_{d+1}, X_e being point e's table read at the new
                                 point's own shift; 0 = off */
    int32_t scheme;           /* rows of the line solve (Section 2.1): RT_SCHEME_FEAUTRIER2 (0), the
                                 second-order equation with second-order end rows (eq. 1);
                                 RT_SCHEME_HERMITE (1), the fourth-order Hermitian rows with
                                 third-order end rows.  Hermitian row d, outer step a, inner step b:
                                 -A' u_{d-1} + (1 + A' + C') u_d - C' u_{d+1}
                                   = al S_{d-1} + (1 - al - ga) S_d + ga S_{d+1},
                                 al = w(a,b), ga = w(b,a), w(x,y) = (x^3 + 2x^2 y - y^3)/(6x(x+y)^2),
                                 A' = 2/(a(a+b)) - al, C' = 2/(b(a+b)) - ga; end row with step t:
                                 (1 + E + 2/t^2) u_0 - (2/t^2) u_1 = S_0 + E I + (S_1 - S_0)/3,
                                 E = (2/t)(1 + t^2/6).  The elimination needs A' >= 0 and C' > 0,
                                 i.e. steps below about 3.46 (e.g. through dtau_max); a line that
                                 breaks this gets u = NaN and latches RT_ERR_STEP.  FP32 tables
                                 need steps above about 1e-18 (2/step^2 stays finite). */
} rt_solve_opts;
enum { RT_SCHEME_FEAUTRIER2 = 0, RT_SCHEME_HERMITE = 1 };
enum { RT_WALK_EXACT = 0, RT_WALK_PADDED = 1, RT_WALK_TWO_PASS = 2 };

/* Scratch needed by rt_solve (u per (origin, pair, frequency), bins). */
rt_status rt_solve_workspace(const rt_dirset* set, int64_t n_origins, int64_t F, const rt_solve_opts* opts,
                             size_t* bytes);

/* J for every listed origin from precomputed ray lists.  u_out, if not NULL,
 * receives u[n_origins][R][F] (dtype of the precision).  Async. */
rt_status rt_solve(const rt_model* model, const rt_dirset* set, const int32_t* origins, int64_t n_origins,
                   const int64_t* ray_off, const int32_t* ray_ids, const double* ray_Z,
                   const void* chi, const void* eta, int32_t dtype, int64_t ld, const rt_freq_grid* grid,
                   const double* I_bc, void* J, void* u_out, const rt_solve_opts* opts,
                   void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ J in one call
 * The whole path for a list of origins -- trace (count, scan, write), sweep and
 * J (eq. 3, eq. 4) -- inside the caller's workspace, the origins taken in
 * chunks whose ray lists fit it.  The origins are put in Morton order of their
 * positions (shared sets; an adaptive set keeps the list order) and cut into
 * consecutive chunks, so each chunk walks one region of the model; within a
 * chunk rays and sweep items run direction by direction over that order
 * (opts->schedule RT_SCHED_SPATIAL or RT_SCHED_DIRECT) or length-binned
 * (RT_SCHED_BINNED); the J rows go back to the caller's list order.  Results
 * are bit-identical to rt_trace_count + rt_trace_write + rt_solve on the whole
 * list: every ray and every (origin, pair) is computed the same way wherever
 * it falls.
 *
 * rt_compute_J_workspace: bytes with which one chunk holds every origin,
 * assuming rays of at most `mean_entries` list entries on average (<= 0: 64).
 * Less workspace is allowed: rt_compute_J then takes as many origins per chunk
 * as the space left for lists admits at the mean ray length of the chunks
 * already traced (a first chunk of at most 1024 origins), recounting a chunk
 * at half the size when its lists do not fit; RT_ERR_CAPACITY when a single
 * origin's rays do not fit, or the workspace is below the fixed part for one
 * origin (about 2R*(4+8+12) + R*F*s + 1 KiB bytes).
 * rt_compute_J: origins device int32 [n_origins] (NULL = 0..n_origins-1);
 * J [n_origins][F] of the precision's dtype; u_out (may be NULL) receives
 * u[n_origins][R][F].  Synchronises `stream` once per chunk (to read the chunk's
 * list length) and once for the Morton order; allocates nothing; everything
 * else is async. */
rt_status rt_compute_J_workspace(const rt_dirset* set, int64_t n_origins, int64_t F, const rt_solve_opts* opts,
                                 double mean_entries, size_t* bytes);
rt_status rt_compute_J(const rt_model* model, const rt_dirset* set, const int32_t* origins, int64_t n_origins,
                       const void* chi, const void* eta, int32_t dtype, int64_t ld, const rt_freq_grid* grid,
                       const double* I_bc, void* J, void* u_out, const rt_solve_opts* opts, void* ws,
                       size_t ws_bytes, void* stream);

/* rt_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments and results as rt_solve without the workspace.  Its scratch (u,
 * unless u_out is given, and the length bins of RT_SCHED_BINNED) is a static
 * 64 MiB device array that each GPU the library runs on holds until the
 * process ends; a call needing more (rt_solve_workspace for the same
 * arguments, with u_out NULL counting u) returns RT_ERR_CAPACITY before
 * launching anything.  The call allocates nothing and never synchronises,
 * except that the first call on a device looks up the scratch's and the error
 * word's addresses (make one call before capturing); the direction set's tables
 * must already be on the device (a shared set uploads them on its first use by
 * any other call, e.g. rt_trace_count; otherwise RT_ERR_STATE).
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * GPU (different streams, or host threads) race and must be serialised by the
 * caller.  Async. */
rt_status rt_solve_noalloc(const rt_model* model, const rt_dirset* set, const int32_t* origins, int64_t n_origins,
                           const int64_t* ray_off, const int32_t* ray_ids, const double* ray_Z, const void* chi,
                           const void* eta, int32_t dtype, int64_t ld, const rt_freq_grid* grid, const double* I_bc,
                           void* J, void* u_out, const rt_solve_opts* opts, void* stream);

/* ------------------------------------------------------------------ plans
 * A plan owns the ray-list buffers for a fixed (model, set, origins) and replays
 * the whole hot path -- trace, (scan, list output), bin, sweep, reduce -- as one
 * HIP graph on the caller's stream.  Creation runs the count pass once to size
 * the lists (synchronises) and allocates; rt_plan_run allocates nothing.  The
 * walk of each run follows opts->walk: by default every ray is walked once and
 * written straight into its slot (the lists' offsets come from the creation-time
 * count); RT_WALK_PADDED walks once into per-ray slots sized by the longest ray
 * and compacts them (when the padded budget allows); RT_WALK_TWO_PASS counts,
 * scans and writes.  A ray that no longer fits its slot (the model's positions
 * changed after creation) latches RT_ERR_CAPACITY. */
typedef struct rt_plan rt_plan;
rt_status rt_plan_create(const rt_model* model, const rt_dirset* set, const int32_t* origins,
                         int64_t n_origins, const void* chi, const void* eta, int32_t dtype, int64_t ld,
                         const rt_freq_grid* grid, const double* I_bc, void* J, const rt_solve_opts* opts,
                         void* stream, rt_plan** out);
/* Replay the plan (async).  use_graph = 0 launches the kernels one by one. */
rt_status rt_plan_run(rt_plan* plan, int32_t use_graph, void* stream);
/* Run the plan eagerly n_runs times on `stream` with HIP events between its
 * stages and return the mean time per stage in ms: stage_ms[6] = {walk (exact
 * write, padded or count), scan, list output (write walk or compaction), bin,
 * sweep, reduce} (scan and list output are ~0 for RT_WALK_EXACT; bin, the
 * queue reset of RT_SCHED_BINNED whose item order a plan builds once when it is
 * configured, is ~0).  Synchronises. */
rt_status rt_plan_profile(rt_plan* plan, int32_t n_runs, double* stage_ms, void* stream);
/* Total ray-list entries, and the plan's device ray lists (borrowed views). */
rt_status rt_plan_info(const rt_plan* plan, int64_t* total_entries, const int64_t** ray_off,
                       const int32_t** ray_ids, const double** ray_Z);
/* Copy the plan's current ray lists into caller buffers (device; sizes
 * n_origins*2R+1, total, total).  Async. */
rt_status rt_plan_copy_rays(const rt_plan* plan, int64_t* ray_off, int32_t* ray_ids, double* ray_Z, void* stream);
/* Copy the per-pair mean intensities of the plan's last run, u[n_origins][R][F]
 * (eq. 3 before the weighted sum; dtype of the precision), into a caller device
 * buffer.  Async. */
rt_status rt_plan_copy_u(const rt_plan* plan, void* u, void* stream);
/* Destroy a plan.  Waits for the device to be idle (as freeing device memory
 * does), then keeps the plan's large buffers (ray lists, padded slots, u; each
 * 64 MiB or more) in a per-device cache of at most 32 GiB, from which later
 * plans of similar size take their buffers instead of allocating: building
 * plan after plan over origin chunks then maps no new memory.  A request that
 * no cached block fits frees the smaller blocks of its device; an allocation
 * that fails releases the cache of its device and retries once.  Memory held
 * by the cache is not available to other allocators (e.g. PyTorch's): call
 * rt_release_cached_memory when the plans are done. */
rt_status rt_plan_destroy(rt_plan* plan);
/* Free every cached buffer (all devices). */
rt_status rt_release_cached_memory(void);
/* Bytes currently held by the cache (all devices). */
rt_status rt_cached_memory(size_t* bytes);
/* Bytes of the large plan buffers (ray lists, padded slots, u) owned by plans
 * not yet destroyed (all devices; the requested sizes). */
rt_status rt_plan_memory(size_t* bytes);

/* Re-capture a plan's graph with other scheduling options (schedule, group,
 * trace_lanes, waves_per_cu, n_bins; precision and threshold stay), reusing its
 * lists and buffers; builds the spatial order or bin workspace on first use.
 * Synchronises `stream`. */
rt_status rt_plan_retune(rt_plan* plan, const rt_solve_opts* opts, void* stream);

/* Autotuner.  On the caller's data, one plan is built and re-captured for
 * nine candidate runs; each run varies the walk's lanes per ray (4, 8, 16) and
 * the sweep's schedule and its parameters: spatial with load group 4 and 8;
 * length-binned persistent with load group 8 at 32 waves per CU and bin edges
 * of 4, 2 and 8 per octave (64, 32 and 128 bins), group 4 at 16 waves per CU
 * (4 per octave, 128 bins) and group 8 at 64 waves per CU (4 per octave, 64
 * bins); direct with group 4 and 8.  The HIP-event stage times (one warm-up,
 * n_runs timed, rt_plan_profile) credit the walk and the sweep separately.
 * The fastest of each goes to *best (other fields from *base, or defaults)
 * unless it beats the library default (spatial, group 4, 4 lanes) by less than
 * 5%, in which case the default stays; the sum of the chosen stage times goes
 * to *best_ms.  With cache_path, a line "<signature> <schedule> <group>
 * <lanes> <waves_per_cu> <bins> <bins_per_octave> <ms>" is appended, and a
 * later call with the same signature (device, P, E, R, origins, F, precision,
 * moving, adaptive, scheme, refinement switches) returns the cached choice
 * without timing.  verbose != 0 prints one line per candidate to stderr.
 * Synchronises, allocates. */
rt_status rt_autotune(const rt_model* model, const rt_dirset* set, const int32_t* origins, int64_t n_origins,
                      const void* chi, const void* eta, int32_t dtype, int64_t ld, const rt_freq_grid* grid,
                      const double* I_bc, void* J, const rt_solve_opts* base, int32_t n_runs,
                      const char* cache_path, int32_t verbose, void* stream, rt_solve_opts* best,
                      double* best_ms);
/* The same search on an existing plan (e.g. a batch's), which is left
 * re-captured with the chosen options; no cache.  Synchronises. */
rt_status rt_autotune_plan(rt_plan* plan, int32_t n_runs, int32_t verbose, void* stream, rt_solve_opts* best,
                           double* best_ms);

/* ------------------------------------------------------------------ many models at once
 * Many independent models of different sizes in one launch: a disjoint union
 * built on the device, so rays never cross from one model into another.  Model
 * k's points take the union ids base_k .. base_k + P_k - 1 (base_k = P_0 + ... +
 * P_{k-1}) in the Morton order of that model's positions, so that points near
 * in space are near in the neighbour records and in the union's [P_total][F]
 * tables, which are gathered from the models' tables row by row.  Positions are
 * not moved and every row of neighbour records keeps the order of the model's
 * own ids (the walk's tie order), so every ray is the model's own (its point ids
 * renamed) and every result is bit-identical to solving each model alone.  The
 * union is traced and solved by one plan (a single HIP graph: table gather,
 * walk, sweep over every model's items in one launch -- length-binned
 * persistent or spatial, as opts says -- J reduction and the scatter of J back
 * to each model's own array).  Origins are every point of the union in union
 * order; the inner plan's ray lists (rt_plan_rays, rt_plan_info) carry union
 * ids and are slotted by union origin.
 *
 * rt_batch_create: models[n_models] (handles on the current device), one
 * uniform direction set for all, chi[k]/eta[k] device [P_k][ld[k]] of `dtype`,
 * one frequency grid and I_bc for all, J[k] device [P_k][F].  Builds the union
 * and the plan, and gathers the tables once (synchronises, allocates); a
 * replay gathers them again, so changes to the models' tables between runs
 * are seen.  rt_batch_run: replay (async;
 * use_graph = 0 launches the steps one by one).  rt_batch_plan: the inner plan
 * over the union (for rt_plan_profile, rt_plan_info, rt_plan_retune,
 * rt_autotune_plan); owned by the batch.  rt_batch_union: the union's point
 * and entry counts.  rt_batch_union_index: index (device int32 [P_total],
 * caller-owned) receives the union id of each model point, index[base_k + i]
 * for point i of model k (async on `stream`).
 * rt_compute_J_batched: create, run once, synchronise, destroy. */
typedef struct rt_batch rt_batch;
rt_status rt_batch_create(int32_t n_models, const rt_model* const* models, const rt_dirset* set,
                          const void* const* chi, const void* const* eta, int32_t dtype, const int64_t* ld,
                          const rt_freq_grid* grid, const double* I_bc, void* const* J, const rt_solve_opts* opts,
                          void* stream, rt_batch** out);
rt_status rt_batch_run(rt_batch* batch, int32_t use_graph, void* stream);
rt_status rt_batch_plan(rt_batch* batch, rt_plan** plan);
rt_status rt_batch_union(const rt_batch* batch, int64_t* points, int64_t* entries);
rt_status rt_batch_union_index(const rt_batch* batch, int32_t* index, void* stream);
rt_status rt_batch_destroy(rt_batch* batch);
rt_status rt_compute_J_batched(int32_t n_models, const rt_model* const* models, const rt_dirset* set,
                               const void* const* chi, const void* const* eta, int32_t dtype, const int64_t* ld,
                               const rt_freq_grid* grid, const double* I_bc, void* const* J,
                               const rt_solve_opts* opts, void* stream);

/* ------------------------------------------------------------------ learned closure
 * A cheap J from the nside = 1 set (6 pairs, Section 2.1.3) plus local optical
 * properties is mapped by a small network to the J of the nside = 8 set (384
 * pairs); points whose predicted error exceeds a bound are re-solved by the
 * plain method (rt_plan_* over the flagged origins) and merged back.  Two
 * features come from the paper's re-meshing section: the relative-difference
 * indicator of eq. 6 and the local element size of eq. 8.
 *
 * Network, fixed shape: 16 inputs (12 features, 4 zero) -> 256 -> 256 -> 256 -> 2,
 * SiLU (z / (1 + exp(-z))) after the three hidden layers, outputs y = (m, s):
 * m predicts log(J_fine / J_coarse), s the log variance of that prediction.
 * Products run on the matrix cores in BF16 with FP32 accumulation: inputs,
 * weights, stored pre-activations z and activations silu(z) are BF16; biases
 * and outputs FP32; the backward signal dz is rounded to BF16 before each
 * product.  FP32 master parameters (layout W1[16][256], b1[256], W2[256][256],
 * b2, W3[256][256], b3, W4[256][2], b4[2], row-major, RT_MLP_NPARAM floats)
 * and Adam moments are owned by the handle; BF16 copies are refreshed after
 * every change of the parameters. */
#define RT_MLP_D_IN 16
#define RT_MLP_WIDTH 256
#define RT_MLP_D_OUT 2
#define RT_MLP_NPARAM 136450
#define RT_CLOSURE_STAT_BLOCKS 1024
typedef struct rt_mlp rt_mlp;
rt_status rt_mlp_num_params(int64_t* n);
/* New network: weights N(0, 2/fan_in) (N(0, 1/fan_in) for the output layer,
 * fan_in 12 for the first), biases 0, Adam state 0.  Synchronises. */
rt_status rt_mlp_create(uint64_t seed, void* stream, rt_mlp** out);
rt_status rt_mlp_destroy(rt_mlp* mlp);
/* Parameters / accumulated gradients as RT_MLP_NPARAM host floats.  Synchronise. */
rt_status rt_mlp_get_params(const rt_mlp* mlp, float* host, void* stream);
rt_status rt_mlp_set_params(rt_mlp* mlp, const float* host, void* stream);
rt_status rt_mlp_get_grads(const rt_mlp* mlp, float* host, void* stream);
rt_status rt_mlp_zero_grad(rt_mlp* mlp, void* stream); /* async */
/* Workspace bytes for n samples: 0 for inference, else the stored
 * pre-activations (3*n*256 BF16) plus the backward's transposed signals and
 * activations (5*256 + 16 rows of n rounded up to 32, BF16) and its FP32
 * partial sums (at most 64 chunks of the W1..W3 gradients, one row of the
 * small gradients per signal-pass workgroup). */
rt_status rt_mlp_workspace(int64_t n, int32_t training, size_t* bytes);
/* Y[i][2] (device f32) = network(X[rows[i]]) for i < n; X device BF16 [*][16]
 * (bit patterns as uint16), rows device int32 or NULL (identity).  keep != 0
 * stores the pre-activations in ws for rt_mlp_backward.  n < 2^31.  Async. */
rt_status rt_mlp_forward(rt_mlp* mlp, const uint16_t* X, const int32_t* rows, int64_t n, float* Y, int32_t keep,
                         void* ws, size_t ws_bytes, void* stream);
/* Adds to the gradients d(sum_i dY[i] . Y[i])/d(params) for the samples of the
 * last keep-forward with the same X, rows, n and ws (dY device f32 [n][2]).
 * Partial sums are added in a fixed order: the result is deterministic for a
 * given n on a given device.  Async. */
rt_status rt_mlp_backward(rt_mlp* mlp, const uint16_t* X, const int32_t* rows, int64_t n, const float* dY,
                          void* ws, size_t ws_bytes, void* stream);
/* Mean Gaussian negative log-likelihood over n samples, per sample
 * 0.5 (exp(-s) (t - m)^2 + s) with t = T[rows[i]] (T device f32, rows as in
 * rt_mlp_forward): dY[i] = its gradient w.r.t. Y[i]; *loss_sum (device f32, may
 * be NULL; caller zeroes it) += the sum of the per-sample losses.  Async. */
rt_status rt_mlp_nll(const float* Y, const float* T, const int32_t* rows, int64_t n, float* dY, float* loss_sum,
                     void* stream);
/* One Adam step on the accumulated gradients (bias-corrected moments,
 * decoupled weight decay wd: w -= lr (m_hat / (sqrt(v_hat) + eps) + wd w)),
 * then the BF16 copies are refreshed.  Gradients are left as they are.  Async. */
rt_status rt_mlp_adam_step(rt_mlp* mlp, float lr, float b1, float b2, float eps, float wd, void* stream);
/* Training schedule of rt_mlp_train.  Step k (the network's k-th Adam step,
 * counted from 0 over its lifetime) draws its batch rows i < batch as
 * splitmix64(seed + (k * batch + i + 1) * 0x9E3779B97F4A7C15) mod N (the
 * SplitMix64 finaliser of Steele, Lea and Flood, 2014), and uses the learning
 * rate lr_final + (lr - lr_final) (1 + cos(pi min(k, total_steps) / total_steps)) / 2. */
typedef struct rt_train_opts {
    int64_t batch;       /* samples per step, 1 .. 2^31 - 1 */
    int64_t total_steps; /* length of the cosine schedule, >= 1 */
    float lr, lr_final;
    float b1, b2, eps, wd; /* Adam, as rt_mlp_adam_step */
    uint64_t seed;
} rt_train_opts;
/* Workspace bytes of rt_mlp_train for the given batch. */
rt_status rt_mlp_train_workspace(int64_t batch, size_t* bytes);
/* n_steps training steps on the samples X (device BF16 [N][16]) with targets T
 * (device f32 [N]): each step draws its rows, runs the keep-forward, the NLL
 * (rt_mlp_nll; *loss_sum, device f32 or NULL, accumulates the per-sample
 * losses, the caller zeroes it), clears the gradients, runs the backward and
 * the Adam step of rt_mlp_adam_step.  One step is captured in a HIP graph and
 * replayed n_steps times on `stream`; the step counter and the learning rate
 * are read on the device, so every replay is the step of its own number.  The
 * same steps taken one call at a time with the same rows and learning rates
 * give the same parameters up to the rounding of the learning rate, which is
 * formed here in FP64 from the FP32 lr and lr_final.  The handle keeps the
 * captured graph and reuses it while X, T, N, opts, loss_sum, ws and ws_bytes
 * stay the same (so ws must stay allocated until the handle's next call or
 * its destruction).  Async; RT_ERR_CAPACITY if ws_bytes is below
 * rt_mlp_train_workspace. */
rt_status rt_mlp_train(rt_mlp* mlp, const uint16_t* X, const float* T, int64_t N, const rt_train_opts* opts,
                       int64_t n_steps, float* loss_sum, void* ws, size_t ws_bytes, void* stream);
/* Features feat[(k*F + f)][16] (device f32) for points p = points[k] (device
 * int32, or NULL for p = k) at frequency f < F: 0 log J1[k][f], 1 log chi,
 * 2 log S (S = eta/chi), 3 and 4 neighbour means of log chi and log S, 5 the
 * neighbour standard deviation of log chi, 6 and 7 max over neighbours n of
 * |(f_p - f_n)/(f_p + f_n)| for chi and S (eq. 6), 8 log L_p with L_p the mean
 * distance to the neighbours (eq. 8), 9 log(chi L_p), 10 freq_x[f] / 5,
 * 11 log(neighbour count); with u (device f32 [n_points][R][F], the coarse
 * solve's per-pair mean intensities, rt_plan_copy_u) 12, 13 and 14 the max,
 * min and standard deviation over the R pairs of log(u_r / J1), else zero;
 * 15 zero.  chi, eta device f32 [P][ld]; J1 device f32 [n_points][F]; freq_x
 * device f32 [F] in Doppler widths.  An id outside 0..P-1 gives a zero row and
 * latches RT_ERR_ARG (rt_sync_status).  Async. */
rt_status rt_closure_features(const rt_model* model, const float* chi, const float* eta, int64_t ld, int64_t F,
                              const float* freq_x, const float* J1, const float* u, int64_t R,
                              const int32_t* points, int64_t n_points, float* feat, void* stream);
/* sums[0..15] = column sums of feat[n][16], sums[16..31] = sums of squares
 * (device f64), summed in a fixed order; partial: device f64 scratch of
 * RT_CLOSURE_STAT_BLOCKS*32.  Async. */
rt_status rt_closure_feature_stats(const float* feat, int64_t n, double* sums, double* partial, void* stream);
/* X[i][c] = bf16((feat[i][c] - mean[c]) * inv_std[c]); mean, inv_std host f32 [16]. Async. */
rt_status rt_closure_normalize(const float* feat, int64_t n, const float* mean, const float* inv_std, uint16_t* X,
                               void* stream);
/* Closure and fallback flags: J[p][f] = J1[p][f] exp(Y[p*F+f][0]) for p < n_points;
 * p is flagged when 0.5 Y[p*F+f][1] > log_bound for some f (log_bound = -inf
 * flags every point, +inf none).  flagged (device int32 [n_points]) receives the
 * flagged positions in unspecified order, *n_flagged (device int32) their count.
 * Async. */
rt_status rt_closure_apply(const float* J1, const float* Y, int64_t n_points, int64_t F, float log_bound, float* J,
                           int32_t* flagged, int32_t* n_flagged, void* stream);
/* Training targets T[i] = log(J_fine[i] / J1[i]) (device f32, n values).  Async. */
rt_status rt_closure_targets(const float* J1, const float* J_fine, int64_t n, float* T, void* stream);
/* J[flagged[k]][f] = J_fine[k][f] for k < n_flagged (J [n_points][F]); a
 * position outside 0..n_points-1 is skipped and latches RT_ERR_ARG.  Async. */
rt_status rt_closure_merge(const float* J_fine, const int32_t* flagged, int64_t n_flagged, int64_t F,
                           int64_t n_points, float* J, void* stream);

/* The standardisation the network's inputs were trained with, x_c = bf16((feat_c
 * - mean[c]) * inv_std[c]) (host [16] each; rt_closure_normalize with these
 * values), kept by the handle for rt_closure_J.  Synchronous, host only. */
rt_status rt_mlp_set_input_norm(rt_mlp* mlp, const float* mean, const float* inv_std);

/* The learned closure from start to end for every point of a model: J1 and
 * the per-pair u of the coarse set by rt_compute_J; per (point, frequency) the
 * features of rt_closure_features (frequency x from the grid's x0 and dx),
 * standardised with the handle's input norm, through the network (points taken
 * 65 536 at a time); J = J1 exp(m) and the fallback flags of rt_closure_apply
 * with log_bound; the flagged points re-solved with the fine set by
 * rt_compute_J and merged into J.  chi, eta device f32 [P][ld]; J device f32
 * [P][F]; flagged device int32 [P] receives the flagged point ids (in no
 * particular order), *n_flagged (host) their count.  The workspace holds the
 * coarse solve, one chunk of inference buffers and the fine J of the flagged
 * points (rt_closure_J_workspace with solve_bytes = 0), plus whatever is left
 * for the two rt_compute_J calls, which chunk their origins to fit it
 * (solve_bytes; e.g. rt_compute_J_workspace of the fine set for a few
 * thousand origins).  RT_ERR_STATE if no input norm was set.  Synchronises
 * (per rt_compute_J chunk, and to read the flag count); allocates nothing. */
rt_status rt_closure_J_workspace(const rt_model* model, const rt_dirset* coarse, int64_t F, size_t solve_bytes,
                                 size_t* bytes);
rt_status rt_closure_J(const rt_model* model, const rt_dirset* coarse, const rt_dirset* fine, const float* chi,
                       const float* eta, int64_t ld, const rt_freq_grid* grid, const double* I_bc, const rt_mlp* mlp,
                       float log_bound, float* J, int32_t* flagged, int64_t* n_flagged, const rt_solve_opts* opts,
                       void* ws, size_t ws_bytes, void* stream);

/* Spatial order of an origin list (device int32 [n], or NULL for 0..n-1):
 * order (host int32 [n]) receives the list positions sorted by the Morton code
 * of the origins' positions on a 2^21 grid over their bounding box.  Splitting
 * a large origin list into chunks along this order keeps each chunk's rays
 * in one region of the model.  Synchronises (reads the positions back). */
rt_status rt_spatial_order(const rt_model* model, const int32_t* origins, int64_t n_origins, int32_t* order,
                           void* stream);

/* ------------------------------------------------------------------ re-meshing indicators
 * For a tracer f (device f64 [P], > 0) on the model's points (Section 2.2.2):
 *   Gf_i  = max over neighbours n of |(f_i - f_n)/(f_i + f_n)|      (eq. 6, in [0, 1])
 *   L_i   = mean over neighbours n of |x_i - x_n|                    (eq. 8)
 *   ell_i = L_i f_small if Gf_i >= G_thres, else L_i f_large         (eq. 7)
 * The paper's parameters (Table 1): AMR f_small 0.90, f_large 2.10, G_thres 0.10;
 * SPH 1.00, 2.15, 0.21.  Gf, L, ell: device f64 [P], each may be NULL.  Async. */
rt_status rt_mesh_indicators(const rt_model* model, const double* f, double f_small, double f_large,
                             double G_thres, double* Gf, double* L, double* ell, void* stream);

/* Ring-scheme HEALPix pixel (Section 2.1.3) of each of n host directions
 * dirs[n][3] (any length) at resolution nside (a power of two up to 2^13), on
 * the host, with the same fixed arithmetic the adaptive sets use. */
rt_status rt_healpix_vec2pix(int32_t nside, const double* dirs, int64_t n, int64_t* pix);

/* Synchronise `stream` and return the error latched by kernels since the last
 * call (RT_ERR_CAPACITY; RT_ERR_NONFINITE; RT_ERR_ARG for an origin id outside
 * 0 .. P-1, whose rays are then empty and whose J row is undefined), then
 * clear it. */
rt_status rt_sync_status(void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
