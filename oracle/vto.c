/*
 * vto.c -- CPU oracle for digital Voronoi, Laguerre and Johnson-Mehl
 * diagrams, following Moulinec, arXiv 2201.13234.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg to check the device library.  No product
 * code path may call it.  It shares nothing with the device library.
 *
 * Build: gcc -std=c99 -O2 -fopenmp -ffp-contract=off -fno-fast-math
 *        (no -march flag, so no fused multiply-add can be emitted).
 *
 * Contents
 *   - keys of Sec. 2 with the distances of App. A (eq. de, eq. dL);
 *   - brute force (Alg. "simple Voronoi algorithm", Sec. 3.1);
 *   - the two-step ball algorithm (Alg. faster_voronoi_algo, Sec. 3.2;
 *     Alg. faster_jmak_algo, Sec. 3.3; the Laguerre variant, Sec. 3.4);
 *   - the cost models that fix the ball size (eq. nstep12_3d, eq. v0_3d,
 *     eq. nstep12_jmak with eq. v').
 */
#include "vto.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Geometry shared by every routine of this file                             */
/* ------------------------------------------------------------------------ */

#define MAXD VTO_MAX_DIM

typedef struct {
    int ndim, kind, periodic, lattice;
    int64_t n[MAXD];
    double L[MAXD];
    double h[MAXD];  /* voxel size L_a / n_a */
    double H[MAXD];  /* half period L_a / 2 */
    double G;        /* Johnson-Mehl growth rate */
    int64_t nvox;
    /* general periods: P[i][a] component a of period vector i; hv[i][a] =
     * P[i][a] / n_i; Pinv the inverse of the matrix with columns P[i] (used
     * only to find which translations can be nearest); rown[i] the norm of
     * row i of Pinv */
    double P[MAXD][MAXD], hv[MAXD][MAXD], Pinv[MAXD][MAXD], rown[MAXD];
} geo_t;

/* Inverse of the d x d matrix M (M[a][i] = component a of column i) by
 * Gauss-Jordan elimination with partial pivoting.  Returns 0 when the matrix
 * is singular to working precision. */
static int invert(int d, double M[MAXD][MAXD], double R[MAXD][MAXD])
{
    double A[MAXD][2 * MAXD];
    int r, c, k;
    double scale = 0.0;
    for (r = 0; r < d; ++r)
        for (c = 0; c < d; ++c) {
            A[r][c] = M[r][c];
            A[r][d + c] = (r == c) ? 1.0 : 0.0;
            if (fabs(M[r][c]) > scale)
                scale = fabs(M[r][c]);
        }
    if (!(scale > 0.0) || !isfinite(scale))
        return 0;
    for (c = 0; c < d; ++c) {
        int piv = c;
        double f;
        for (r = c + 1; r < d; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c]))
                piv = r;
        if (!(fabs(A[piv][c]) > 1e-12 * scale))
            return 0;
        if (piv != c)
            for (k = 0; k < 2 * d; ++k) {
                double t = A[c][k];
                A[c][k] = A[piv][k];
                A[piv][k] = t;
            }
        f = A[c][c];
        for (k = 0; k < 2 * d; ++k)
            A[c][k] /= f;
        for (r = 0; r < d; ++r) {
            if (r == c)
                continue;
            f = A[r][c];
            for (k = 0; k < 2 * d; ++k)
                A[r][k] -= f * A[c][k];
        }
    }
    for (r = 0; r < d; ++r)
        for (c = 0; c < d; ++c)
            R[r][c] = A[r][d + c];
    return 1;
}

static void geo_init(geo_t* g, const vto_problem* p)
{
    int a;
    memset(g, 0, sizeof *g);
    g->ndim = p->ndim;
    g->kind = p->kind;
    g->periodic = p->periodic ? 1 : 0;
    g->G = p->growth;
    g->lattice = p->lattice ? 1 : 0;
    g->nvox = 1;
    if (g->lattice) {
        int i, b;
        double M[MAXD][MAXD];
        for (i = 0; i < p->ndim; ++i)
            for (b = 0; b < p->ndim; ++b) {
                g->P[i][b] = p->periods[i * p->ndim + b];
                g->hv[i][b] = g->P[i][b] / (double)p->n[i];
                M[b][i] = g->P[i][b];
            }
        if (invert(p->ndim, M, g->Pinv))
            for (i = 0; i < p->ndim; ++i) {
                double r2 = 0.0;
                for (b = 0; b < p->ndim; ++b)
                    r2 += g->Pinv[i][b] * g->Pinv[i][b];
                g->rown[i] = sqrt(r2);
            }
    }
    for (a = 0; a < MAXD; ++a) {
        if (a < p->ndim) {
            g->n[a] = p->n[a];
            g->L[a] = p->L[a];
            g->h[a] = p->L[a] / (double)p->n[a];
            g->H[a] = 0.5 * p->L[a];
        } else {
            g->n[a] = 1;
            g->L[a] = 1.0;
            g->h[a] = 1.0;
            g->H[a] = 0.5;
        }
        g->nvox *= g->n[a];
    }
}

/* Centre of voxel i along an axis: the paper's x(k) (Sec. 3.1) read as the
 * centre of the cell [i*h, (i+1)*h). */
static double voxel_centre(const geo_t* g, int a, int64_t i)
{
    return ((double)i + 0.5) * g->h[a];
}

/* Signed coordinate difference s - x along axis a.  With periodic
 * boundaries this is the minimum-image difference of App. A:
 * y - x - N((y - x)/L) L with N(y) = floor(y + 1/2), the quotient taken
 * exactly.  Because s and x lie in [0, L), |s - x| < L and the correction
 * is a single subtraction or addition of L, which is exact (Sterbenz). */
static double axis_delta(const geo_t* g, int a, double s, double x)
{
    double d = s - x;
    if (g->periodic) {
        if (d >= g->H[a])
            d = d - g->L[a];
        else if (d < -g->H[a])
            d = d + g->L[a];
    }
    return d;
}

/* A periodic site coordinate brought into the unit cell [0, L): the
 * L-periodic distance of App. A (eq. L-distance_def) does not change when a
 * point moves by a whole period.  fmod is exact; the one rounding is r + L
 * for r < 0, and a sum that rounds up to L is the point 0 of the next
 * period. */
static double cell_coord(double c, double L)
{
    double r = fmod(c, L);
    if (r < 0.0) {
        r = r + L;
        if (r >= L)
            r = 0.0;
    }
    return r + 0.0; /* -0.0 -> +0.0 */
}

/* The sites the routines below work on: the caller's array, or for periodic
 * boundaries a copy with every coordinate brought into the unit cell.
 * Returns NULL when the copy cannot be allocated; release with
 * release_sites. */
static const double* prepare_sites(const geo_t* g, int64_t nsites, const double* coords)
{
    double* c;
    int64_t i;
    if (!g->periodic || g->lattice)
        return coords;
    c = (double*)malloc((size_t)nsites * (size_t)g->ndim * sizeof(double));
    if (!c)
        return NULL;
    for (i = 0; i < nsites * g->ndim; ++i)
        c[i] = cell_coord(coords[i], g->L[i % g->ndim]);
    return c;
}

static void release_sites(const double* sites, const double* coords)
{
    if (sites != coords)
        free((void*)sites);
}

/* The key the diagram minimises at point x for site s (Sec. 2):
 *   squared distance q = d0^2 + T, T = d1^2 then T + d2^2, ... (eq. de /
 *                    eq. dL, squared; in 3D q = d0^2 + (d1^2 + d2^2))
 *   Voronoi:      q                              (eq. Voronoi_Cell; the
 *                                                 squared distance is allowed
 *                                                 by the remark of Sec. 3.1)
 *   Laguerre:     q - w_s                        (power distance, Sec. 2.3)
 *   Johnson-Mehl: t_s + sqrt(q) / G              (eq. JMAK2)              */
/* Squared distance between e = s - x shifted by the translation k (the
 * definition of eq. L-distance_def for one k), summed as in site_key. */
static double lattice_q(const geo_t* g, const double* e, const int64_t* k)
{
    double d[MAXD] = {0.0}, T, q;
    int a, i;
    for (a = 0; a < g->ndim; ++a) {
        double o = (double)k[0] * g->P[0][a];
        for (i = 1; i < g->ndim; ++i)
            o = o + (double)k[i] * g->P[i][a];
        d[a] = e[a] + o;
    }
    if (g->ndim == 1)
        return d[0] * d[0];
    T = d[1] * d[1];
    for (a = 2; a < g->ndim; ++a)
        T = T + d[a] * d[a];
    q = d[0] * d[0] + T;
    return q;
}

/* General periods: the minimum of lattice_q over every translation k.  Any
 * k that can reach the minimum satisfies |k_i - g_i| <= |row i of Pinv| *
 * |d(k0)| with g = Pinv (x - s) and k0 = rint(g), so only the box of those k
 * (widened for rounding) is searched. */
static double lattice_min_q(const geo_t* g, const double* s, const double* x)
{
    double e[MAXD], gv[MAXD], q0, D0, best;
    int64_t k0[MAXD], lo[MAXD], hi[MAXD], k[MAXD];
    int a, i;
    for (a = 0; a < g->ndim; ++a)
        e[a] = s[a] - x[a];
    for (i = 0; i < g->ndim; ++i) {
        double acc = 0.0;
        for (a = 0; a < g->ndim; ++a)
            acc -= g->Pinv[i][a] * e[a];
        gv[i] = acc;
        k0[i] = (int64_t)rint(acc);
    }
    q0 = lattice_q(g, e, k0);
    D0 = sqrt(q0);
    for (i = 0; i < g->ndim; ++i) {
        double r = g->rown[i] * D0 * (1.0 + 0x1p-20) + 0x1p-30 * (1.0 + fabs(gv[i]));
        lo[i] = (int64_t)ceil(gv[i] - r);
        hi[i] = (int64_t)floor(gv[i] + r);
        if (lo[i] > k0[i])
            lo[i] = k0[i];
        if (hi[i] < k0[i])
            hi[i] = k0[i];
        k[i] = lo[i];
    }
    best = q0;
    for (;;) {
        double q = lattice_q(g, e, k);
        if (q < best)
            best = q;
        for (i = 0; i < g->ndim; ++i) {
            if (++k[i] <= hi[i])
                break;
            k[i] = lo[i];
        }
        if (i == g->ndim)
            break;
    }
    return best;
}

static double site_key(const geo_t* g, const double* s, double prm, const double* x)
{
    double q;
    if (g->lattice) {
        q = lattice_min_q(g, s, x);
        if (g->kind == VTO_LAGUERRE)
            return q - prm;
        if (g->kind == VTO_JOHNSON_MEHL)
            return prm + sqrt(q) / g->G;
        return q;
    }
    double d0 = axis_delta(g, 0, s[0], x[0]);
    if (g->ndim == 1) {
        q = d0 * d0;
    } else {
        double d1 = axis_delta(g, 1, s[1], x[1]);
        double T = d1 * d1;
        int a;
        for (a = 2; a < g->ndim; ++a) {
            double da = axis_delta(g, a, s[a], x[a]);
            T = T + da * da;
        }
        q = d0 * d0 + T;
    }
    if (g->kind == VTO_LAGUERRE)
        return q - prm;
    if (g->kind == VTO_JOHNSON_MEHL)
        return prm + sqrt(q) / g->G;
    return q;
}

static int resolve_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    return nthreads < 1 ? 1 : nthreads;
}

int vto_max_threads(void) { return resolve_threads(0); }

/* ------------------------------------------------------------------------ */
/* Validation                                                                */
/* ------------------------------------------------------------------------ */

int vto_validate(const vto_problem* p, int64_t nsites, const double* coords,
                 const double* param)
{
    int a;
    int64_t s;
    if (!p || p->ndim < 1 || p->ndim > MAXD)
        return VTO_ERR_INVALID;
    if (p->kind < VTO_VORONOI || p->kind > VTO_JOHNSON_MEHL)
        return VTO_ERR_INVALID;
    if (nsites < 1 || nsites > 2147483647LL || !coords)
        return VTO_ERR_INVALID;
    if (p->kind != VTO_VORONOI && !param)
        return VTO_ERR_INVALID;
    if (p->kind == VTO_JOHNSON_MEHL && !(p->growth >= VTO_SCALE_MIN && p->growth <= VTO_SCALE_MAX))
        return VTO_ERR_INVALID;
    if (p->lattice) {
        geo_t g;
        int i;
        if (!p->periodic)
            return VTO_ERR_INVALID;
        for (a = 0; a < p->ndim * p->ndim; ++a)
            if (!(fabs(p->periods[a]) <= VTO_SCALE_MAX))
                return VTO_ERR_INVALID;
        for (i = 0; i < p->ndim; ++i) {
            double len2 = 0.0, len;
            for (a = 0; a < p->ndim; ++a)
                len2 += p->periods[i * p->ndim + a] * p->periods[i * p->ndim + a];
            len = sqrt(len2);
            if (!(len >= VTO_SCALE_MIN && len <= VTO_SCALE_MAX))
                return VTO_ERR_INVALID;
        }
        for (a = 0; a < p->ndim; ++a)
            if (p->n[a] < 1 || p->n[a] > 2147483647LL)
                return VTO_ERR_INVALID;
        geo_init(&g, p);
        for (a = 0; a < p->ndim; ++a)
            if (!(g.rown[a] > 0.0 && isfinite(g.rown[a])))
                return VTO_ERR_INVALID; /* singular period matrix */
    }
    for (a = 0; a < p->ndim; ++a) {
        if (p->n[a] < 1 || p->n[a] > 2147483647LL)
            return VTO_ERR_INVALID;
        if (!p->lattice && !(p->L[a] >= VTO_SCALE_MIN && p->L[a] <= VTO_SCALE_MAX))
            return VTO_ERR_INVALID;
    }
    for (s = 0; s < nsites; ++s) {
        for (a = 0; a < p->ndim; ++a) {
            double c = coords[s * p->ndim + a];
            if (p->lattice) {
                if (!(fabs(c) <= VTO_SCALE_MAX))
                    return VTO_ERR_INPUT;
                continue;
            }
            if (p->periodic ? !isfinite(c) : !(c >= 0.0 && c < p->L[a]))
                return VTO_ERR_INPUT;
        }
        if (p->kind != VTO_VORONOI && !(fabs(param[s]) <= VTO_SCALE_MAX))
            return VTO_ERR_INPUT;
    }
    return VTO_OK;
}

/* ------------------------------------------------------------------------ */
/* Cost models (Sec. 3.2.3, 3.3.2, 3.4)                                      */
/* ------------------------------------------------------------------------ */

static double unit_ball_volume(int d)
{
    /* omega_d = pi^(d/2) / Gamma(d/2 + 1) */
    const double pi = 3.14159265358979323846;
    return pow(pi, 0.5 * d) / tgamma(0.5 * d + 1.0);
}

static double domain_volume(const vto_problem* p)
{
    double V = 1.0;
    int a;
    for (a = 0; a < p->ndim; ++a)
        V *= p->L[a];
    return V;
}

static double sum_sq_lengths(const vto_problem* p)
{
    double S = 0.0;
    int a;
    for (a = 0; a < p->ndim; ++a)
        S += p->L[a] * p->L[a];
    return S;
}

double vto_v0_fraction(int64_t nsites)
{
    /* eq. v0_3d: v0 / V = 1 - (1/N_s)^(1/(N_s - 1)) */
    double N = (double)nsites;
    if (nsites <= 1)
        return 1.0;
    return 1.0 - pow(1.0 / N, 1.0 / (N - 1.0));
}

/* Volume of the ball of site s at level tau (the "investigation ball"):
 *   Voronoi      radius r0 = sqrt(tau)
 *   Johnson-Mehl radius r_s = G (t0 - t_s)^+          (eq. rs JM, tau = t0)
 *   Laguerre     radius r_s = sqrt(G (t0 - t_s)^+)    (eq. rs Laguerre),
 *                written with w_s = -G t_s and tau = G t0 as
 *                r_s^2 = (tau + w_s)^+                                    */
static double ball_radius(const vto_problem* p, double prm, double tau)
{
    if (p->kind == VTO_VORONOI)
        return tau > 0.0 ? sqrt(tau) : 0.0;
    if (p->kind == VTO_LAGUERRE) {
        double r2 = tau + prm;
        return r2 > 0.0 ? sqrt(r2) : 0.0;
    }
    {
        double dt = tau - prm;
        return dt > 0.0 ? p->growth * dt : 0.0;
    }
}

double vto_cost_model(const vto_problem* p, int64_t nsites, const double* param,
                      double tau)
{
    double V = domain_volume(p);
    double Nv = 1.0, Ns = (double)nsites;
    double wd = unit_ball_volume(p->ndim);
    int a;
    for (a = 0; a < p->ndim; ++a)
        Nv *= (double)p->n[a];
    if (p->kind == VTO_VORONOI) {
        /* eq. nstep12_3d with v'_s = v0 (eq. nstep1b):
         * E = N_s N_v (v0/V + (1 - v0/V)^N_s) */
        double r = tau > 0.0 ? sqrt(tau) : 0.0;
        double f = wd * pow(r, p->ndim) / V;
        if (f > 1.0)
            f = 1.0;
        return Ns * Nv * (f + pow(1.0 - f, Ns));
    } else {
        /* eq. nstep12_jmak: E = N_v sum_s v'_s/V + N_s N_v prod_s (1 - v'_s/V)
         * with v'_s = min(V, v_s) (eq. v'); the product is taken as the
         * exponential of a sum of logarithms so that it does not underflow. */
        double step1 = 0.0, logp = 0.0;
        int64_t s;
        for (s = 0; s < nsites; ++s) {
            double r = ball_radius(p, param[s], tau);
            double f = wd * pow(r, p->ndim) / V;
            if (f > 1.0)
                f = 1.0;
            step1 += f;
            logp += (f >= 1.0) ? -INFINITY : log1p(-f);
        }
        return Nv * step1 + Ns * Nv * exp(logp);
    }
}

double vto_choose_tau(const vto_problem* p, int64_t nsites, const double* param)
{
    double lo, hi, span;
    int it;
    if (nsites <= 1)
        return INFINITY; /* eq. v0_3d divides by N_s - 1 = 0: one ball covers everything */
    if (p->kind == VTO_VORONOI) {
        /* eq. v0_3d, then v0 = omega_d r0^d */
        double v0 = vto_v0_fraction(nsites) * domain_volume(p);
        double r0 = pow(v0 / unit_ball_volume(p->ndim), 1.0 / p->ndim);
        return r0 * r0;
    }
    if (p->kind == VTO_JOHNSON_MEHL) {
        /* Sec. 3.3.2: t0 lies in [min t, min t + sqrt(sum L^2)/(2G)]
         * (periodic) or [min t, min t + sqrt(sum L^2)/G] (non-periodic). */
        double tmin = param[0];
        int64_t s;
        for (s = 1; s < nsites; ++s)
            if (param[s] < tmin)
                tmin = param[s];
        span = sqrt(sum_sq_lengths(p)) / p->growth;
        if (p->periodic)
            span *= 0.5;
        lo = tmin;
        hi = tmin + span;
    } else {
        /* Sec. 3.4: t0 in [min t, min t + sum L^2/(4G)] (periodic) or
         * [min t, min t + sum L^2/G] (non-periodic); with G t_s = -w_s and
         * tau = G t0 this is tau in [-max w, -max w + sum L^2 / 4] or
         * [-max w, -max w + sum L^2]. */
        double wmax = param[0];
        int64_t s;
        for (s = 1; s < nsites; ++s)
            if (param[s] > wmax)
                wmax = param[s];
        span = sum_sq_lengths(p);
        if (p->periodic)
            span *= 0.25;
        lo = -wmax;
        hi = -wmax + span;
    }
    /* Dichotomy on the slope of the cost model (Sec. 3.3.2 asks for "a
     * dichotomy method"): compare the model just left and right of the
     * midpoint and keep the half that holds the smaller value. */
    for (it = 0; it < 80; ++it) {
        double mid = 0.5 * (lo + hi);
        double eps = (hi - lo) * 1e-4;
        double fl = vto_cost_model(p, nsites, param, mid - eps);
        double fr = vto_cost_model(p, nsites, param, mid + eps);
        if (fl <= fr)
            hi = mid + eps;
        else
            lo = mid - eps;
        if (!(hi - lo > 1e-12 * (fabs(lo) + fabs(hi) + 1e-300)))
            break;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------------ */
/* Brute force (Alg. simple Voronoi algorithm, Sec. 3.1)                     */
/* ------------------------------------------------------------------------ */

/* Brute force at one voxel: every site in ascending order, strict "<". */
static void brute_voxel(const geo_t* g, int64_t nsites, const double* coords,
                        const double* param, const double* x, int32_t* lab,
                        double* key)
{
    double D = INFINITY;
    int32_t I = -1;
    int64_t s;
    for (s = 0; s < nsites; ++s) {
        double k = site_key(g, coords + s * g->ndim, param ? param[s] : 0.0, x);
        if (k < D) {
            D = k;
            I = (int32_t)s;
        }
    }
    *lab = I;
    *key = D;
}

/* Centre of the voxel with index vector k: the orthogonal reading per axis,
 * or for general periods x_a = sum_i (k_i + 1/2) (L_ia / n_i) in order. */
static void voxel_at(const geo_t* g, const int64_t* k, double* x)
{
    int a, i;
    if (!g->lattice) {
        for (a = 0; a < g->ndim; ++a)
            x[a] = voxel_centre(g, a, k[a]);
        return;
    }
    for (a = 0; a < g->ndim; ++a) {
        double acc = ((double)k[0] + 0.5) * g->hv[0][a];
        for (i = 1; i < g->ndim; ++i)
            acc = acc + ((double)k[i] + 0.5) * g->hv[i][a];
        x[a] = acc;
    }
}

static void voxel_point(const geo_t* g, int64_t lin, double* x)
{
    int64_t k[MAXD];
    int a;
    for (a = 0; a < g->ndim; ++a) {
        k[a] = lin % g->n[a];
        lin /= g->n[a];
    }
    voxel_at(g, k, x);
}

int vto_brute(const vto_problem* p, int64_t nsites, const double* coords,
              const double* param, int nthreads, int32_t* labels, double* keys_out)
{
    geo_t g;
    int64_t v;
    const double* sites;
    int rc = vto_validate(p, nsites, coords, param);
    if (rc != VTO_OK)
        return rc;
    if (!labels)
        return VTO_ERR_INVALID;
    geo_init(&g, p);
    sites = prepare_sites(&g, nsites, coords);
    if (!sites)
        return VTO_ERR_NOMEM;
    nthreads = resolve_threads(nthreads);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (v = 0; v < g.nvox; ++v) {
        double x[MAXD], k;
        int32_t l;
        voxel_point(&g, v, x);
        brute_voxel(&g, nsites, sites, param, x, &l, &k);
        labels[v] = l;
        if (keys_out)
            keys_out[v] = k;
    }
    release_sites(sites, coords);
    return VTO_OK;
}

int vto_label_points(const vto_problem* p, int64_t nsites, const double* coords,
                     const double* param, int64_t npts, const int64_t* vox,
                     int nthreads, int32_t* labels, double* keys_out)
{
    geo_t g;
    int64_t i;
    const double* sites;
    int rc = vto_validate(p, nsites, coords, param);
    if (rc != VTO_OK)
        return rc;
    if (npts < 0 || (npts > 0 && (!vox || !labels)))
        return VTO_ERR_INVALID;
    geo_init(&g, p);
    for (i = 0; i < npts; ++i) {
        int a;
        for (a = 0; a < p->ndim; ++a)
            if (vox[MAXD * i + a] < 0 || vox[MAXD * i + a] >= g.n[a])
                return VTO_ERR_INVALID;
    }
    sites = prepare_sites(&g, nsites, coords);
    if (!sites)
        return VTO_ERR_NOMEM;
    nthreads = resolve_threads(nthreads);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (i = 0; i < npts; ++i) {
        double x[MAXD], k;
        int32_t l;
        voxel_at(&g, vox + MAXD * i, x);
        brute_voxel(&g, nsites, sites, param, x, &l, &k);
        labels[i] = l;
        if (keys_out)
            keys_out[i] = k;
    }
    release_sites(sites, coords);
    return VTO_OK;
}

/* ------------------------------------------------------------------------ */
/* Two-step ball algorithm (Sec. 3.2.2, 3.3.1, 3.4)                          */
/* ------------------------------------------------------------------------ */

/* Voxel indices along axis a whose centres may lie within distance R of
 * coordinate s: a conservative index box, one voxel wider on each side than
 * the ball so that rounding of the key cannot leave a member outside.
 * Writes the (wrapped, in periodic mode) indices to out and returns their
 * count.  Ball membership itself is decided later by the key. */
static int64_t axis_box(const geo_t* g, int a, double s, double R, int64_t* out)
{
    int64_t n = g->n[a], lo, hi, i, cnt = 0;
    if (!(R < 2.0 * g->L[a])) {
        for (i = 0; i < n; ++i)
            out[i] = i;
        return n;
    }
    lo = (int64_t)floor((s - R) / g->h[a] - 0.5) - 1;
    hi = (int64_t)ceil((s + R) / g->h[a] - 0.5) + 1;
    if (g->periodic) {
        if (hi - lo + 1 >= n) {
            for (i = 0; i < n; ++i)
                out[i] = i;
            return n;
        }
        for (i = lo; i <= hi; ++i)
            out[cnt++] = ((i % n) + n) % n;
        return cnt;
    }
    if (lo < 0)
        lo = 0;
    if (hi > n - 1)
        hi = n - 1;
    for (i = lo; i <= hi; ++i)
        out[cnt++] = i;
    return cnt;
}

int vto_tessellate(const vto_problem* p, int64_t nsites, const double* coords,
                   const double* param, double tau, int nthreads,
                   int32_t* labels, double* keys_out, vto_stats* stats)
{
    geo_t g;
    double* D;
    const double* sites;
    int64_t n_step1 = 0, n_box = 0, n_out = 0, nidx = 0;
    int outer, rc, failed = 0, a;
    rc = vto_validate(p, nsites, coords, param);
    if (rc != VTO_OK)
        return rc;
    if (!labels)
        return VTO_ERR_INVALID;
    geo_init(&g, p);
    if (g.lattice) {
        /* general periods: the brute-force definition (the index boxes of
         * step 1 assume orthogonal periods) */
        rc = vto_brute(p, nsites, coords, param, nthreads, labels, keys_out);
        if (rc == VTO_OK && stats) {
            stats->tau = NAN;
            stats->n_step1 = 0;
            stats->n_box = 0;
            stats->n_out = g.nvox;
            stats->n_step2 = g.nvox * nsites;
        }
        return rc;
    }
    outer = g.ndim - 1; /* threads own slabs along the slowest axis */
    nthreads = resolve_threads(nthreads);
    for (a = 0; a < g.ndim; ++a)
        nidx += g.n[a];

    /* Initialisation: the level tau (eq. v0_3d or the t0 search), D = inf. */
    if (isnan(tau))
        tau = vto_choose_tau(p, nsites, param);
    sites = prepare_sites(&g, nsites, coords);
    if (!sites)
        return VTO_ERR_NOMEM;
    D = keys_out ? keys_out : (double*)malloc((size_t)g.nvox * sizeof(double));
    if (!D) {
        release_sites(sites, coords);
        return VTO_ERR_NOMEM;
    }

#pragma omp parallel num_threads(nthreads) reduction(+ : n_step1, n_box, n_out)
    {
        int T = 1, t = 0;
        int64_t o0, o1, v, s, plane = 1;
        int64_t* idx;
#ifdef _OPENMP
        T = omp_get_num_threads();
        t = omp_get_thread_num();
#endif
        int ax;
        o0 = g.n[outer] * t / T;
        o1 = g.n[outer] * (t + 1) / T;
        for (ax = 0; ax < outer; ++ax)
            plane *= g.n[ax];
        idx = (int64_t*)malloc((size_t)nidx * sizeof(int64_t));
        if (!idx) {
#pragma omp atomic write
            failed = 1;
        } else {
            for (v = o0 * plane; v < o1 * plane; ++v) {
                D[v] = INFINITY;
                labels[v] = -1;
            }

            /* Step 1: for s = 1..N_s, every voxel of the ball of s takes s if
             * its key is strictly below D. */
            for (s = 0; s < nsites; ++s) {
                const double* sp = sites + s * g.ndim;
                double prm = param ? param[s] : 0.0;
                double R = ball_radius(p, prm, tau);
                int64_t* box[MAXD];
                int64_t cnt[MAXD], pos[MAXD];
                int64_t off = 0, c;
                int b, empty = 0;
                if (tau == -INFINITY)
                    break;
                if (p->kind == VTO_VORONOI && !(tau >= 0.0))
                    break;
                if (p->kind == VTO_LAGUERRE && !(tau + prm >= 0.0))
                    continue;
                if (p->kind == VTO_JOHNSON_MEHL && !(tau >= prm))
                    continue;
                /* the index box of the ball, axis by axis */
                for (b = 0; b < g.ndim; ++b) {
                    box[b] = idx + off;
                    cnt[b] = axis_box(&g, b, sp[b], R, box[b]);
                    off += g.n[b];
                    pos[b] = 0;
                    if (cnt[b] == 0)
                        empty = 1;
                }
                if (empty)
                    continue;
                /* every voxel of the box: axis 0 innermost, the others by an
                 * odometer over their index lists */
                for (;;) {
                    int64_t jo = box[outer][pos[outer]];
                    if (g.ndim == 1 || (jo >= o0 && jo < o1)) {
                        double x[MAXD];
                        int64_t base = 0, stride = 1;
                        for (b = 0; b < g.ndim; ++b) {
                            if (b > 0)
                                base += box[b][pos[b]] * stride;
                            x[b] = voxel_centre(&g, b, box[b][pos[b]]);
                            stride *= g.n[b];
                        }
                        for (c = 0; c < cnt[0]; ++c) {
                            int64_t lin = base + box[0][c];
                            double k;
                            if (g.ndim == 1 && (box[0][c] < o0 || box[0][c] >= o1))
                                continue;
                            x[0] = voxel_centre(&g, 0, box[0][c]);
                            k = site_key(&g, sp, prm, x);
                            ++n_box;
                            if (k <= tau) { /* the voxel is inside the ball */
                                ++n_step1;
                                if (k < D[lin]) {
                                    D[lin] = k;
                                    labels[lin] = (int32_t)s;
                                }
                            }
                        }
                    }
                    for (b = 1; b < g.ndim; ++b) {
                        if (++pos[b] < cnt[b])
                            break;
                        pos[b] = 0;
                    }
                    if (b >= g.ndim)
                        break;
                }
            }

            /* Step 2: voxels outside every ball go through the brute-force
             * loop. */
            for (v = o0 * plane; v < o1 * plane; ++v) {
                if (labels[v] == -1) {
                    double x[MAXD];
                    ++n_out;
                    voxel_point(&g, v, x);
                    brute_voxel(&g, nsites, sites, param, x, &labels[v], &D[v]);
                }
            }
            free(idx);
        }
    }
    release_sites(sites, coords);
    if (!keys_out)
        free(D);
    if (failed)
        return VTO_ERR_NOMEM;
    if (stats) {
        stats->tau = tau;
        stats->n_step1 = n_step1;
        stats->n_box = n_box;
        stats->n_out = n_out;
        stats->n_step2 = n_out * nsites;
    }
    return VTO_OK;
}
