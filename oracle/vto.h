/*
 * vto.h -- CPU oracle for digital images of Voronoi, Laguerre and
 * Johnson-Mehl diagrams (Moulinec, arXiv 2201.13234).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the
 * smoke check and the benchmark's CPU baseline can check the device library
 * against an independent, plain implementation of the paper's method.  No
 * product code path may link, load or call it.  It shares no code, header,
 * table or constant with the device library.
 *
 * What it computes (paper Sec. 2 and Sec. 3):
 *   For every voxel k of an n_0 x ... x n_{d-1} grid (1 <= d <= 6; the paper
 *   states the method for any dimension, Sec. 3) on the box
 *   Omega = [0,L_0) x ... x [0,L_{d-1}), the label I(k) is the index of the
 *   site that minimises the diagram's key at the voxel centre x(k):
 *     Voronoi      key = q                      (squared distance, Sec. 3.1)
 *     Laguerre     key = q - w_s                (power distance, Sec. 2.3)
 *     Johnson-Mehl key = t_s + sqrt(q) / v      (arrival time, eq. JMAK2)
 *   q is the squared Euclidean distance (App. A, eq. de) or, for periodic
 *   boundaries, the squared L-periodic distance (App. A, eq. dL).  Ties go
 *   to the lowest site index, which is what the paper's strict "<" test over
 *   sites taken in ascending order produces.
 *
 * Fixed readings of points the paper leaves open (each also listed in the
 * design notes of the repository):
 *   - voxel centre: x_a = ((double)i_a + 0.5) * (L_a / n_a), i_a 0-based;
 *   - minimum image: delta = s_a - x_a; if delta >= L_a/2 subtract L_a, else
 *     if delta < -L_a/2 add L_a.  This is the paper's nearest-integer
 *     function N(y) = floor(y + 1/2) applied to the exact quotient
 *     delta / L_a (never to a rounded one);
 *   - q = d0*d0 + T with T = d1*d1, then T = T + d2*d2, ... over the
 *     remaining axes in order (3D: d0*d0 + (d1*d1 + d2*d2); 2D: d0*d0 + d1*d1;
 *     1D: d0*d0), each operation rounded once in IEEE binary64 (build with
 *     -ffp-contract=off);
 *   - periodic boundaries: a site coordinate may be any finite number (App. A
 *     defines the L-periodic distance for points outside the unit cell); it
 *     is first brought into [0, L_a) by r = fmod(c, L_a), which is exact,
 *     then r + L_a if r < 0, and 0 if that sum rounds up to L_a;
 *   - general period vectors L_i (App. A, eq. L-distance_def; lattice = 1):
 *     the grid covers the cell {sum_i alpha_i L_i, alpha in [0,1)^d}; voxel k
 *     is centred at x_a = sum_i ((double)k_i + 0.5) * (L_ia / n_i), summed
 *     over i in order; the squared distance to site s is the minimum over
 *     all integer k of the folded sum of d_a^2 with
 *     d_a = (s_a - x_a) + (k_0 L_0a + k_1 L_1a + ...), summed in order.
 *     Sites are Cartesian, any finite value, not reduced.  With a diagonal
 *     matrix and sites inside the cell this equals the orthogonal reading
 *     bit for bit.  Only the brute-force definition is used (the two-step
 *     algorithm's index boxes assume orthogonal periods);
 *   - labels are 0-based.
 *
 * Precision: all arithmetic is IEEE binary64 with round-to-nearest, no
 * contraction into fused multiply-add, correctly rounded sqrt and division.
 */
#ifndef VTO_H
#define VTO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { VTO_VORONOI = 0, VTO_LAGUERRE = 1, VTO_JOHNSON_MEHL = 2 };
enum { VTO_MAX_DIM = 6 };

/* Return codes (same numeric values as the device library's codes). */
enum { VTO_OK = 0, VTO_ERR_INVALID = 1, VTO_ERR_NOMEM = 2, VTO_ERR_INPUT = 5 };

/* Problem statement of Sec. 3 (list at the top of the section). */
typedef struct {
    int32_t ndim;      /* 1 .. VTO_MAX_DIM */
    int32_t kind;      /* VTO_VORONOI, VTO_LAGUERRE or VTO_JOHNSON_MEHL */
    int32_t periodic;  /* 1: L-periodic distance (App. A); 0: Euclidean */
    int32_t lattice;   /* 1: general period vectors in `periods` (needs periodic = 1) */
    int64_t n[VTO_MAX_DIM]; /* voxels per axis; axis 0 fastest in memory; entries >= ndim ignored */
    double  L[VTO_MAX_DIM]; /* domain lengths; entries >= ndim ignored */
    double  growth;    /* Johnson-Mehl growth rate G (= v) > 0; ignored otherwise */
    double  periods[VTO_MAX_DIM * VTO_MAX_DIM]; /* lattice = 1: periods[i*ndim + a] is
                                                   component a of period vector L_i */
} vto_problem;

/* Operation counters of the two-step algorithm (Sec. 3.2.3, Figs. voro4/fdl). */
typedef struct {
    double  tau;       /* level used in step 1 (r0^2, G*t0 or t0, see vto_tessellate) */
    int64_t n_step1;   /* voxels found inside a ball during step 1 (key <= tau) */
    int64_t n_box;     /* keys evaluated in step 1 over the conservative index boxes */
    int64_t n_out;     /* voxels still unassigned after step 1 */
    int64_t n_step2;   /* keys evaluated in step 2 (= n_out * N_s) */
} vto_stats;

/* Supported scale.  The problem statement (Sec. 3) puts no bound on the
 * lengths, times or weights; binary64 does.  Lengths L_a, the growth rate G
 * and the period vectors' entries and lengths lie in [VTO_SCALE_MIN,
 * VTO_SCALE_MAX]; |w_s|, |t_s| and, with period vectors, |site coordinates|
 * are at most VTO_SCALE_MAX.  Then every squared distance and key is finite
 * and the rounding margins the tests rely on stay normal numbers. */
#define VTO_SCALE_MAX 0x1p200
#define VTO_SCALE_MIN 0x1p-200

/* Checks the problem scalars and every site (finite; inside [0,L_a) unless
 * the boundaries are periodic; parameter within the scale bound).  Returns
 * VTO_OK, VTO_ERR_INVALID (bad scalars) or VTO_ERR_INPUT (bad site data). */
int vto_validate(const vto_problem* p, int64_t nsites, const double* coords,
                 const double* param);

/* Step 0 of the accelerated algorithms: the level tau that minimises the
 * paper's cost model.
 *   Voronoi      tau = r0^2 with v0/V = 1 - N^(-1/(N-1))      (eq. v0_3d)
 *   Johnson-Mehl tau = t0 minimising eq. nstep12_jmak over the interval of
 *                Sec. 3.3.2, found by dichotomy
 *   Laguerre     tau = G*t0 with G*t_s = -w_s (App. B), minimising the same
 *                model over the interval given at the end of Sec. 3.4
 * Returns +inf for a single site (the model's N-1 = 0 case). */
double vto_choose_tau(const vto_problem* p, int64_t nsites, const double* param);

/* Expected number of key evaluations of the two steps at level tau:
 * eq. nstep12_3d for Voronoi (v'_s = v0), eq. nstep12_jmak with
 * v'_s = min(V, v_s) (eq. v') for Johnson-Mehl and Laguerre. */
double vto_cost_model(const vto_problem* p, int64_t nsites, const double* param,
                      double tau);

/* Ball volume fraction of eq. v0_3d: v0/V = 1 - (1/N)^(1/(N-1)). */
double vto_v0_fraction(int64_t nsites);

/* The accelerated two-step algorithm (Alg. faster_voronoi_algo, Alg.
 * faster_jmak_algo and its Laguerre variant, Sec. 3.2-3.4), generalised to a
 * level tau: step 1 takes the sites in ascending order and, for every voxel
 * whose key is <= tau (the ball of the site), keeps the site if its key is
 * strictly below the current D; step 2 runs the brute-force loop on the
 * voxels left without a site.  tau = NaN selects vto_choose_tau().
 * coords: [nsites][ndim] host array; param: [nsites] (w_s for Laguerre, t_s
 * for Johnson-Mehl; NULL for Voronoi).  labels: prod(n) int32 output.
 * keys_out (nullable): prod(n) doubles, the minimum key per voxel (the image
 * D of the paper).  stats (nullable) receives the operation counts.
 * nthreads <= 0 uses every available OpenMP thread. */
int vto_tessellate(const vto_problem* p, int64_t nsites, const double* coords,
                   const double* param, double tau, int nthreads,
                   int32_t* labels, double* keys_out, vto_stats* stats);

/* Brute-force algorithm (Alg. simple Voronoi algorithm and its variants for
 * the other keys): every voxel against every site. */
int vto_brute(const vto_problem* p, int64_t nsites, const double* coords,
              const double* param, int nthreads, int32_t* labels,
              double* keys_out);

/* Brute force at selected voxels only: vox is [npts][VTO_MAX_DIM] voxel
 * indices (entries >= ndim ignored); writes label and minimum key per point. */
int vto_label_points(const vto_problem* p, int64_t nsites, const double* coords,
                     const double* param, int64_t npts, const int64_t* vox,
                     int nthreads, int32_t* labels, double* keys_out);

/* Number of OpenMP threads a call with nthreads <= 0 would use. */
int vto_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif /* VTO_H */
