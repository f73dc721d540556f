/*
 * vtess.h -- C ABI of the MI355X library that computes digital images of
 * Voronoi, Laguerre and Johnson-Mehl diagrams (Moulinec, arXiv 2201.13234).
 *
 * Problem (Sec. 3, list at the top of the section): a regular grid of
 * n_0 x n_1 [x n_2] voxels covers the box Omega = [0,L_0) x [0,L_1) [x [0,L_2)].
 * Every voxel gets the 0-based index of the site that minimises, at the
 * voxel centre x_a = (i_a + 1/2) * L_a / n_a,
 *   Voronoi       q                 (squared distance; cells of eq. Voronoi_Cell)
 *   Laguerre      q - w_s           (power distance of Sec. 2.3, w_s = r_s^2)
 *   Johnson-Mehl  t_s + sqrt(q) / v (arrival time of eq. JMAK2, growth rate v)
 * where q is the squared Euclidean distance (App. A, eq. de) or, with periodic
 * boundaries, the squared L-periodic distance (App. A, eq. dL).  The result is
 * bit-identical to brute force in IEEE binary64 with
 *   d_a = s_a - x_a, minimum image d_a -= L_a if d_a >= L_a/2,
 *   d_a += L_a if d_a < -L_a/2, q = d0*d0 + (d1*d1 + d2*d2) (3D) or
 *   d0*d0 + d1*d1 (2D), every operation rounded once (no fused multiply-add),
 * and ties go to the lowest site index (the paper's strict '<' over sites in
 * ascending order, Alg. "simple Voronoi algorithm").
 *
 * Conventions
 *  - All device work is asynchronous on the caller's HIP stream (passed as
 *    void*, a hipStream_t; NULL is the default stream).
 *  - Device pointers: coords, param, labels and status arrays are device
 *    memory owned by the caller, who keeps them alive until the stream has
 *    completed the call.  The library owns its scratch and vt_bins objects.
 *  - Errors are return codes; nothing is thrown across the ABI.  Errors in
 *    scalars are reported before any launch.  Bad coordinates or parameters
 *    are found on the device: that job's labels become -1 and its status word
 *    (if given) becomes VT_ERR_INPUT once the stream has run the call.
 *  - Threading: a vt_ctx is used by one host thread at a time.
 *  - Scale (Sec. 3 leaves it open; the bound keeps every squared distance, key
 *    and rounding margin a finite normal binary64 number): lengths L_a, the
 *    growth rate v and the entries and row lengths of period vectors lie in
 *    [VT_SCALE_MIN, VT_SCALE_MAX] (else VT_ERR_INVALID before any launch);
 *    |w_s|, |t_s| and, with period vectors, |coordinates| are at most
 *    VT_SCALE_MAX (else VT_ERR_INPUT from the device).
 */
#ifndef VTESS_H
#define VTESS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { VT_VORONOI = 0, VT_LAGUERRE = 1, VT_JOHNSON_MEHL = 2 } vt_kind;
typedef enum { VT_NONPERIODIC = 0, VT_PERIODIC = 1 } vt_bc;
typedef enum {
    VT_OK = 0,
    VT_ERR_INVALID = 1, /* bad scalar argument (dims, lengths, growth, null pointer) */
    VT_ERR_NOMEM = 2,   /* device or host allocation failed */
    VT_ERR_HIP = 3,     /* a HIP runtime call failed (see vt_last_error) */
    VT_ERR_BUSY = 4,    /* resource limit of the call exceeded (e.g. batch too large) */
    VT_ERR_INPUT = 5    /* bad site coordinates or parameters, found on the device */
} vt_status;

#define VT_SCALE_MAX 0x1p200  /* about 1.6e60 */
#define VT_SCALE_MIN 0x1p-200 /* about 6.2e-61 */

typedef struct vt_ctx vt_ctx;   /* device, scratch pool, tuning table */
typedef struct vt_bins vt_bins; /* one job's sites binned on the device */

/* One diagram to label (problem statement of Sec. 3). */
typedef struct {
    int32_t ndim;        /* 2 or 3 */
    int32_t kind;        /* vt_kind */
    int32_t bc;          /* vt_bc */
    int32_t reserved;    /* must be 0 */
    int64_t n[3];        /* voxels per axis, axis 0 fastest in memory; n[2] ignored in 2D */
    double  L[3];        /* domain lengths in [VT_SCALE_MIN, VT_SCALE_MAX]; L[2] ignored in 2D */
    double  growth;      /* Johnson-Mehl growth rate v in [VT_SCALE_MIN, VT_SCALE_MAX] (G of
                          * eq. JMAK2); ignored otherwise */
    int64_t nsites;      /* 1 .. 2^31 - 1 */
    const double* coords;/* device, [nsites][ndim] binary64: in [0, L_a) for non-periodic
                          * boundaries; any finite value for periodic ones (brought into
                          * [0, L_a) by an exact fmod, then + L_a if negative, 0 if that
                          * sum rounds to L_a: App. A defines the L-periodic distance for
                          * points outside the unit cell) */
    const double* param; /* device, [nsites]: Laguerre w_s, Johnson-Mehl t_s, |value| <=
                          * VT_SCALE_MAX; NULL for Voronoi */
    int32_t* labels;     /* device, prod(n) int32 written by the call (x fastest) */
    double*  keys;       /* device, prod(n) binary64 or NULL: the winning key per voxel (the
                          * distance image: q for Voronoi, q - w for Laguerre, t + sqrt(q)/v
                          * for Johnson-Mehl; Sec. 3 notes the squared distance map as a
                          * by-product), bit-identical to the key that chose the label;
                          * NaN where the job's input is bad */
} vt_job;

/* General dimension (1 .. VT_MAX_DIM axes; the method is stated for any
 * dimension in Sec. 3).  Fields as in vt_job, with
 *   q = d0*d0 + T,  T = d1*d1, then T = T + d2*d2, ... over the remaining
 *   axes in order (3D: d0*d0 + (d1*d1 + d2*d2); 2D: d0*d0 + d1*d1; 1D:
 *   d0*d0), each operation rounded once. */
#define VT_MAX_DIM 6
enum { VT_ND_GENERIC = 1 }; /* flags: use the general kernel for 2 and 3 axes as well */
typedef struct {
    int32_t ndim;        /* 1 .. VT_MAX_DIM */
    int32_t kind;        /* vt_kind */
    int32_t bc;          /* vt_bc */
    int32_t flags;       /* 0 or VT_ND_GENERIC */
    int64_t n[VT_MAX_DIM]; /* voxels per axis, axis 0 fastest in memory; entries >= ndim ignored */
    double  L[VT_MAX_DIM]; /* domain lengths > 0; entries >= ndim ignored */
    double  growth;      /* Johnson-Mehl growth rate v > 0; ignored otherwise */
    int64_t nsites;      /* 1 .. 2^31 - 1 */
    const double* coords;/* device, [nsites][ndim], as for vt_job */
    const double* param; /* device, [nsites] or NULL for Voronoi */
    int32_t* labels;     /* device, prod(n) int32 */
    double*  keys;       /* device, prod(n) binary64 or NULL: the winning key per voxel */
    const double* periods; /* host, NULL or [ndim][ndim]: periods[i*ndim + a] is component a of
                          * period vector L_i (App. A, eq. L-distance_def; needs bc =
                          * VT_PERIODIC, L is then ignored).  The grid covers the cell
                          * {sum_i alpha_i L_i, alpha in [0,1)^d}: voxel k is centred at
                          * x_a = sum_i ((double)k_i + 0.5) * (L_ia / n_i), summed over i in
                          * order, and q is the minimum over integer translations k of the
                          * folded sum of d_a^2 with d_a = (s_a - x_a) + (k_0 L_0a + k_1 L_1a
                          * + ...), summed in order.  Sites are Cartesian, any finite value.
                          * A diagonal matrix and sites inside the cell give the orthogonal
                          * result bit for bit.  VT_ERR_INVALID for a singular or non-finite
                          * matrix.  Always runs the general kernel. */
} vt_job_nd;

/* Creates a context on HIP device `device`.  Reads a tuning cache from the
 * file named by the environment variable VT_TUNE_CACHE if it is set.  A
 * context owns one scratch arena that each call reuses: give each context
 * one stream (or order its calls), and one host thread at a time. */
vt_status vt_create(int device, vt_ctx** out);
void vt_destroy(vt_ctx* ctx);

/* Grows the context's scratch to at least `bytes` now (synchronising the
 * device once), so that later calls that fit never have to grow it, which
 * would synchronise the device in the middle of queued work.  For serving
 * loops.  VT_ERR_NOMEM if the allocation fails. */
vt_status vt_reserve(vt_ctx* ctx, size_t bytes);

/* Plain single-diagram path: labels every voxel of job with the lowest
 * index of the sites that minimise its key (the problem of Sec. 3, keys of
 * Sec. 2 and App. A as above; the ineffective Johnson-Mehl sites of Sec. 3.3
 * are dropped first, labels unchanged).  Bins the sites (counting sort into a
 * uniform bin grid), then labels voxel tiles with bound-based pruning and an
 * exact evaluation of the survivors.  status_dev (nullable): one
 * device int32, set to VT_OK or VT_ERR_INPUT by the kernels.  May grow the
 * context's scratch, which synchronises the device.  Calls on one context
 * share its scratch (each call's kernels also clear words for the next call),
 * so order them: one stream, or synchronise between streams.  A call captured
 * into a graph clears its own words; its replays are valid while no later
 * call has grown the context's scratch. */
vt_status vt_tessellate(vt_ctx* ctx, const vt_job* job, int32_t* status_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the plain
 * path of vt_tessellate, same kernels and same results, run on a static
 * scratch array of VT_NOALLOC_SCRATCH_BYTES per device instead of the
 * context's arena.  It calls no hipMalloc, hipFree or other allocating
 * routine.  The array is allocated when the library's code object is loaded
 * on a device and held until the process ends; vt_create looks up its address
 * on its device.  A job whose binning arrays need more (about 44 bytes per
 * site plus 8 per bin and 16 per region of four tiles, e.g. some 1.2 million
 * uniform sites) gets VT_ERR_BUSY before any launch.  Every call on one device
 * shares that array, whatever its context: calls that overlap on one GPU
 * (other streams, other threads) race and give wrong labels, so order them.
 * The kernels clear what must start at zero.  Other arguments and errors as
 * for vt_tessellate. */
#define VT_NOALLOC_SCRATCH_BYTES (64u << 20)
vt_status vt_tessellate_noalloc(vt_ctx* ctx, const vt_job* job, int32_t* status_dev, void* stream);

/* Any dimension from 1 to VT_MAX_DIM.  Jobs with 2 or 3 axes and no period
 * vectors go through vt_tessellate unless flags holds VT_ND_GENERIC; the
 * others (and those with the flag) run the general kernel: a counting sort of the sites into a
 * d-dimensional bin grid, then per tile of at most 256 voxels a search over
 * rings of bins until the sites beyond them provably lose, and a
 * lexicographic (key, index) minimum over the remaining candidates.  Same
 * results, status word, errors and scratch behaviour as vt_tessellate
 * (n_a in [1, 2^30], at most 2^40 voxels, else VT_ERR_INVALID). */
vt_status vt_tessellate_nd(vt_ctx* ctx, const vt_job_nd* job, int32_t* status_dev, void* stream);

/* Many diagrams (each the problem of Sec. 3, as for vt_tessellate), of any
 * sizes, kinds and boundaries: one segmented binning pass over all of them, then one labelling launch per group of jobs that
 * share kind, dimension and tile configuration (each group runs a kernel
 * compiled for it, one workgroup per region of the group's jobs).  status_dev (nullable): njobs device int32, one
 * per job, in the order of `jobs`.  A job with bad sites gets -1 labels and
 * VT_ERR_INPUT without affecting the others.  Johnson-Mehl jobs first drop
 * from their bins the sites that provably never win (a site s whose
 * nucleation another site's grain reaches first: t_r + |s - r| / v < t_s by
 * more than the rounding margin); labels are unchanged by it. */
vt_status vt_tessellate_batch(vt_ctx* ctx, const vt_job* jobs, int32_t njobs,
                              int32_t* status_dev, void* stream);

/* Bins one job's sites into device memory owned by the returned object,
 * which stays resident until vt_bins_free.  The job's coords/param buffers
 * are read only by this call; labels is kept as the output buffer of later
 * vt_label_batch calls.  status_dev (nullable) as for vt_tessellate. */
vt_status vt_bins_build(vt_ctx* ctx, const vt_job* job, vt_bins** out,
                        int32_t* status_dev, void* stream);

/* Labels the jobs behind n resident bin objects (one launch per group, as
 * for vt_tessellate_batch), writing each into the labels buffer
 * given at vt_bins_build.  status_dev
 * (nullable): n device int32 (VT_ERR_INPUT for jobs whose binning flagged bad
 * input, else VT_OK). */
vt_status vt_label_batch(vt_ctx* ctx, vt_bins* const* bins, int32_t n,
                         int32_t* status_dev, void* stream);

/* Releases a bin object after the work queued on `stream` that uses it. */
vt_status vt_bins_free(vt_ctx* ctx, vt_bins* bins, void* stream);

/* Picks the launch plan per job class (dimension, kind, boundary, size class
 * floor(log2(voxels) / 2), density class floor(log2(voxels / sites))) from the
 * sample jobs.  For each class it times the built-in plan, then every tile
 * configuration with bins of 1.0, 1.2, 1.4, 1.6 and 2.0 mean spacings (and,
 * for Laguerre, a first gather box of one or two bins); a round runs each
 * sample alone (vt_tessellate) and all of the class's samples in one
 * vt_tessellate_batch call, best of three.  A candidate replaces the built-in
 * plan only if its round is at least 3 % faster.  The chosen plans stay in the
 * context (later calls of every path use them) and, if cache_path is not
 * NULL, go to that file as JSON with both times ("ms", "default_ms").  The
 * samples' label buffers are overwritten.  Synchronous. */
vt_status vt_autotune(vt_ctx* ctx, const vt_job* samples, int32_t n, const char* cache_path);

/* Loads a tuning cache written by vt_autotune. */
vt_status vt_load_tuning(vt_ctx* ctx, const char* cache_path);

/* Forces the tile configuration and bin-size factor of later calls
 * (tile_cfg < 0 and bin_factor <= 0 restore the tuned/default choice).
 * Tile configurations (voxels, x first): 3D 0 = 8x16x8, 1 = 8x8x8,
 * 2 = 8x4x4, 3 = 4x4x4; 2D 0 = 32x32, 1 = 32x16, 2 = 16x8, 3 = 8x8.  By default
 * the tile shrinks as the sites get denser (voxels per site).  The bin factor
 * (bin side over the mean site spacing) applies to vt_tessellate_nd too. */
vt_status vt_set_params(vt_ctx* ctx, int32_t tile_cfg, double bin_factor);

/* Bins per axis and tile configuration the next call would use for job,
 * after the same scalar checks as vt_tessellate (VT_ERR_INVALID on failure;
 * nothing is launched and no device memory is touched).  ctx may be NULL: the
 * default plan, without tuning cache or forced parameters.  Output pointers
 * are host memory and may be NULL. */
vt_status vt_plan(vt_ctx* ctx, const vt_job* job, int32_t* bins_per_axis3,
                  int32_t* tile_cfg, double* bin_factor);

/* The same for vt_tessellate_nd's general kernel: bins per axis and tile
 * voxels per axis (host arrays of job->ndim entries, or NULL).  ctx may be
 * NULL.  Jobs that vt_tessellate_nd would send to vt_tessellate are planned
 * as general-kernel jobs here. */
vt_status vt_plan_nd(vt_ctx* ctx, const vt_job_nd* job, int32_t* bins_per_axis, int32_t* tile_voxels);

/* Device-numerics probe: sqrt_out[i] = sqrt(x[i]) and div_out[i] = x[i] / den[i]
 * computed by the same binary64 operations the labelling kernels use, so that
 * a test can check them against correctly rounded host results (the keys of
 * eq. JMAK2 need an IEEE square root and division).  All four arrays are
 * device memory of n doubles. */
vt_status vt_numerics_probe(vt_ctx* ctx, const double* x, const double* den, double* sqrt_out,
                            double* div_out, int64_t n, void* stream);

/* Order-sensitive checksum of a label image, for checking results without
 * copying them to the host (serving, benchmarks).  Adds
 *     sum over i < n of (labels[i] + 3) * ((i * 48271 + 97) mod P),
 * taken mod P = 2^31 - 1 per workgroup (at most 1024 of them), to *acc_dev (a
 * device uint64 that the caller zeroes).  The
 * checksum is *acc_dev mod P once the stream reaches this point.  labels is a
 * device int32 array of n entries; nothing is allocated.  VT_ERR_INVALID for
 * n < 0 or NULL pointers with n > 0. */
vt_status vt_label_digest(vt_ctx* ctx, const int32_t* labels, int64_t n, unsigned long long* acc_dev,
                          void* stream);

/* Phase timing of the plain path, for benchmarks.  While enabled, every
 * vt_tessellate call records four HIP events on its own stream: before the
 * binning kernels, before the main labelling kernel, after it, and after the
 * overflow kernel that labels the tiles the main kernel left over.
 * vt_profile_read waits for the recorded events, returns the summed
 * milliseconds of the three phases and the number of calls recorded, and
 * clears the record.  Any output pointer may be NULL. */
vt_status vt_profile_enable(vt_ctx* ctx, int32_t enable);
vt_status vt_profile_read(vt_ctx* ctx, double* bin_ms, double* label_ms, double* overflow_ms,
                          int64_t* calls);

const char* vt_status_string(vt_status s);
/* Detail text of the last error of the calling thread. */
const char* vt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VTESS_H */
