// label_core.h -- device code of the labelling kernels, shared by the
// single-diagram kernels (label_kernel.hip) and the persistent batch
// kernels (label_batch.hip).  What is computed and how is described at the
// top of label_kernel.hip.
#pragma once

#include "vt_internal.h"

namespace vt {

namespace {

constexpr int NW = 4;          // wavefronts per workgroup = tiles per region
constexpr int NT = NW * WAVE;  // threads per workgroup
constexpr int CAP_R = 576;     // region candidate capacity (LDS)
constexpr int CAP_S = 64;      // tile candidate capacity (LDS, per wavefront)
constexpr int CAP_F = 64;      // fallback per-tile capacity (LDS, per wavefront)

// flags: wrap code per axis in bits 2a..2a+1 (0 none, 1 subtract L, 2 add L),
// bit 6 = some axis needs a per-voxel minimum-image test.
constexpr int FL_GENERIC = 64;
// Evaluation records: every squared distance of the site to the tile's voxel
// centres is at least 2^-500, so the Johnson-Mehl keys may use sqrt_refined.
constexpr int FL_SQRT_FAST = 256;

enum { KV = 0, KL = 1, KJM = 2, KJD = 3 };  // Johnson-Mehl: multiply by exact 1/v, or divide

// Dominance references (the candidates with the smallest upper bounds): six
// for Voronoi, four for Laguerre and Johnson-Mehl (measured against 4 to 12;
// each reference costs a test per candidate).
constexpr int r_dom(int kind) { return kind == KV ? 6 : 4; }

// A tile list entry refers to its site record in the region list through the
// position stored above the flags (cm.y >> 8).
struct TileLds {
    double4 cg[CAP_S];  // minimum image {x, y, z} over the tile and e = |image|^2 (- w for Laguerre)
    double2 cq[CAP_S];  // {min, max} distance to the tile box
    int2 cm[CAP_S];     // {site index, flags}
    union {
        int ci[CAP_S];      // region-list positions that passed the lower-bound test, then
        unsigned ck[CAP_S]; // 32-bit ranking keys (upper bound, then site index)
    };
};

// After pruning, tiles whose lanes all cover the same 8 x positions keep
// their survivors as evaluation records, written over the (then dead) list
// arrays: the squared x differences are the same for every lane, so they are
// computed once per survivor instead of once per lane.
constexpr int XRUN = 8;
struct EvalRec {
    double dx2[XRUN];  // squared x difference at the 8 x positions (wrap code applied)
    double y, z, p;    // site y, z and parameter
    int idx, flags;    // site index, flags (wrap codes of y and z are used)
};
constexpr int CAP_E = (int)(sizeof(TileLds) / sizeof(EvalRec));

struct RegionLds {
    double4 rs[CAP_R];
    int ri[CAP_R];
    int rf[CAP_R];  // wrap code per axis of the site's image in the gather box (2 bits per axis)
    int wsum[NW];
    double wred[NW];
};

struct FallbackLds {
    double4 cs[CAP_F];
    double4 cg[CAP_F];
    double2 cb[CAP_F];  // {lower, upper} bound of the key over the tile box
    double2 cq[CAP_F];
    int2 cm[CAP_F];
    unsigned ck[CAP_F];
    int bcnt[WAVE];
    int bsrc[WAVE];
};

struct Smem {
    struct {
        RegionLds reg;
        TileLds tile[NW];
    } r;
};

struct TileBox {
    double lo[3], hi[3];  // box of voxel centres
};

// A job's record in device memory that no kernel writes while labelling runs
// (one record for the single-job kernels, the job table for batches), read
// through the constant address space: the labelling code then loads each
// field with scalar loads where it needs it, instead of holding a copy of the
// whole record in registers.  (Measured faster than passing the record as a
// kernel argument: M2 0.646 against 0.666 ms, M4 0.648 against 0.692 ms.)
using ConstJob = const __attribute__((address_space(4))) JobDev;

__device__ inline const JobDev& job_ref(const JobDev* jobs, int j)
{
    return *(const JobDev*)&((ConstJob*)jobs)[j];
}

struct JobConst {
    double M;        // pruning margin
    double pmax, pmin;
    double v, rv;    // growth rate and its reciprocal
    double sqrtL2;   // sqrt(sum L_a^2)
};

// ------------------------------------------------------------------ helpers

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int wrap_code(double d, double H) { return d >= H ? 1 : (d < -H ? 2 : 0); }
__device__ inline double code_off(int c, double L) { return c == 1 ? -L : (c == 2 ? L : 0.0); }
__device__ inline double min_image(double d, double H, double L)
{
    return d >= H ? d - L : (d < -H ? d + L : d);
}

// q = e / d and r = e % d for 0 <= e < 2^30, 1 <= d, through a float
// reciprocal with an exact integer correction step.
__device__ inline int divmod_small(int e, int d, float rd, int& r)
{
    int q = (int)(((float)e + 0.5f) * rd);
    r = e - q * d;
    while (r < 0) {
        --q;
        r += d;
    }
    while (r >= d) {
        ++q;
        r -= d;
    }
    return q;
}

// Periodic bin index in [0, nb) for unwrapped b in [-2 nb, 3 nb).
__device__ inline int wrap_bin(int b, int nb)
{
    b = b < 0 ? b + nb : b;
    b = b < 0 ? b + nb : b;
    b = b >= nb ? b - nb : b;
    b = b >= nb ? b - nb : b;
    return b;
}

__device__ inline double from_ordered(unsigned long long u)
{
    unsigned long long b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)b);
}

__device__ inline double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmin(v, __shfl_xor(v, o));
    return v;
}

__device__ inline int wave_inclusive_add(int v, int lane)
{
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(v, o);
        if (lane >= o)
            v += t;
    }
    return v;
}

__device__ inline unsigned long long lanes_below(int lane)
{
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ inline int block_excl_scan(int v, int& total, int* wsum, int tid)
{
    const int lane = tid & (WAVE - 1), w = tid / WAVE;
    const int inc = wave_inclusive_add(v, lane);
    if (lane == WAVE - 1)
        wsum[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int s = wsum[k];
        off += k < w ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

__device__ inline double block_min(double v, double* wred, int tid)
{
    v = wave_min(v);
    if ((tid & (WAVE - 1)) == 0)
        wred[tid / WAVE] = v;
    __syncthreads();
    double r = wred[0];
#pragma unroll
    for (int k = 1; k < NW; ++k)
        r = fmin(r, wred[k]);
    __syncthreads();
    return r;
}

__device__ inline double block_max(double v, double* wred, int tid)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    if ((tid & (WAVE - 1)) == 0)
        wred[tid / WAVE] = v;
    __syncthreads();
    double r = wred[0];
#pragma unroll
    for (int k = 1; k < NW; ++k)
        r = fmax(r, wred[k]);
    __syncthreads();
    return r;
}

// dist_key with sqrt_refined (for q >= 2^-500 only).
template <int KIND>
__device__ inline double dist_key_fast(double q, double p, double v, double rv)
{
    if (KIND == KJM)
        return p + sqrt_refined(q) * rv;
    return p + sqrt_refined(q) / v;
}

template <int KIND>
__device__ inline double dist_key(double q, double p, double v, double rv)
{
    if (KIND == KV)
        return q;
    if (KIND == KL)
        return q - p;
    if (KIND == KJM)
        return p + sqrt(q) * rv;
    return p + sqrt(q) / v;
}

template <int KIND>
__device__ inline JobConst job_const(const JobDev& J, int dim)
{
    JobConst C;
    double sumL2 = 0.0;
    for (int a = 0; a < dim; ++a)
        sumL2 += J.L[a] * J.L[a];
    C.sqrtL2 = sqrt(sumL2);
    C.v = J.growth;
    C.rv = J.rgrowth;
    C.pmax = C.pmin = 0.0;
    if (KIND != KV) {
        C.pmax = from_ordered(J.pbound[0]);
        C.pmin = -from_ordered(J.pbound[1]);
    }
    const double pabs = fmax(fabs(C.pmax), fabs(C.pmin));
    const double scale = (KIND == KV) ? sumL2 : (KIND == KL) ? sumL2 + 2.0 * pabs : C.sqrtL2 * C.rv + 2.0 * pabs;
    C.M = scale * 0x1p-36;
    return C;
}

// Voxel-centre box of voxels [v0, ve] (ve clipped to the grid).
template <int DIM>
__device__ inline TileBox make_box(const JobDev& J, const int* v0, const int* ve)
{
    TileBox B;
    for (int a = 0; a < 3; ++a) {
        if (a < DIM) {
            B.lo[a] = ((double)v0[a] + 0.5) * J.h[a];
            B.hi[a] = ((double)ve[a] + 0.5) * J.h[a];
        } else {
            B.lo[a] = B.hi[a] = 0.0;
        }
    }
    return B;
}

// Bounds of site s over box B: wrap flags, lower/upper bound of the key,
// min/max distance, and the linear-form record {image, e} used by the
// dominance test (image = minimum image of s over the box, e = |image|^2,
// minus w for Laguerre).
template <int KIND, int DIM>
__device__ inline void box_bounds(const JobDev& J, const JobConst& C, const TileBox& B, bool periodic,
                                  const double4& s, int& flags, double& lb, double& ub, double& dmn,
                                  double& dmx, double4& g)
{
    const double sc[3] = {s.x, s.y, s.z};
    double sg3[3] = {0.0, 0.0, 0.0};
    double qmin = 0.0, qmax = 0.0, e = 0.0;
    flags = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double sg = sc[a], dmin, dmax;
        bool gen = false;
        if (periodic) {
            const int c1 = wrap_code(sc[a] - B.lo[a], J.H[a]);
            const int c2 = wrap_code(sc[a] - B.hi[a], J.H[a]);
            if (c1 == c2) {
                flags |= c1 << (2 * a);
                sg = sc[a] + code_off(c1, J.L[a]);
            } else {
                gen = true;
            }
        }
        if (gen) {
            // The wrap flips inside the box: it contains the point half a
            // period from the site, where the periodic distance peaks at
            // L/2, so over the box the distance is smallest at an end (unless
            // the box spans half a period itself).
            flags |= FL_GENERIC;
            dmin = 0.0;
            if (B.hi[a] - B.lo[a] < J.H[a])
                dmin = fmin(fabs(min_image(sc[a] - B.lo[a], J.H[a], J.L[a])),
                            fabs(min_image(sc[a] - B.hi[a], J.H[a], J.L[a])));
            dmax = J.H[a];
        } else {
            dmin = fmax(0.0, fmax(B.lo[a] - sg, sg - B.hi[a]));
            dmax = fmax(fabs(sg - B.lo[a]), fabs(sg - B.hi[a]));
        }
        sg3[a] = sg;
        e += sg * sg;
        qmin += dmin * dmin;
        qmax += dmax * dmax;
    }
    if (KIND == KV) {
        lb = qmin;
        ub = qmax;
        dmn = dmx = 0.0;
    } else if (KIND == KL) {
        lb = qmin - s.w;
        ub = qmax - s.w;
        e -= s.w;
        dmn = dmx = 0.0;
    } else {
        dmn = sqrt(qmin);
        dmx = sqrt(qmax);
        lb = s.w + dmn * C.rv;
        ub = s.w + dmx * C.rv;
    }
    g = make_double4(sg3[0], sg3[1], sg3[2], e);
}

// Coordinates of a site's image given its wrap codes (2 bits per axis).
// `wrapped` is false when no bin of the gather box lies outside the grid: the
// codes are then all zero and the image is the site itself.
template <int DIM>
__device__ inline void site_image(const JobDev& J, const double4& s, int code, bool wrapped, double* sg)
{
    const double sc[3] = {s.x, s.y, s.z};
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        sg[a] = sc[a];
    if (wrapped) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int c = (code >> (2 * a)) & 3;
            sg[a] = sc[a] + (double)((c >> 1) - (c & 1)) * J.L[a];
        }
    }
}

// Upper bound of the key over box B through a given image of the site.  Any
// image bounds the minimum-image distance from above, so this is valid for
// every gather box.
template <int KIND, int DIM>
__device__ inline double image_upper(const JobConst& C, const TileBox& B, const double* sg, double p)
{
    double qmax = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double dmax = fmax(fabs(sg[a] - B.lo[a]), fabs(sg[a] - B.hi[a]));
        qmax += dmax * dmax;
    }
    if (KIND == KV)
        return qmax;
    if (KIND == KL)
        return qmax - p;
    return p + sqrt(qmax) * C.rv;
}

// Lower bound of the key over box B through the site's minimum image sg.
template <int KIND, int DIM>
__device__ inline double image_lower(const JobConst& C, const TileBox& B, const double* sg, double p)
{
    double qmin = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double dmin = fmax(0.0, fmax(B.lo[a] - sg[a], sg[a] - B.hi[a]));
        qmin += dmin * dmin;
    }
    if (KIND == KV)
        return qmin;
    if (KIND == KL)
        return qmin - p;
    return p + sqrt(qmin) * C.rv;
}

// image_lower that also returns the minimum distance to the box (Johnson-Mehl
// only; 0 otherwise).
template <int KIND, int DIM>
__device__ inline double image_lower_d(const JobConst& C, const TileBox& B, const double* sg, double p, double& dmin)
{
    double qmin = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double d = fmax(0.0, fmax(B.lo[a] - sg[a], sg[a] - B.hi[a]));
        qmin += d * d;
    }
    dmin = 0.0;
    if (KIND == KV)
        return qmin;
    if (KIND == KL)
        return qmin - p;
    dmin = sqrt(qmin);
    return p + dmin * C.rv;
}

// Lower-bound test of a site over box B against the level thr (key <= thr is
// possible), without square roots: Johnson-Mehl compares the squared minimum
// distance with ((thr - t) v)^2, widened by a relative 2^-40 that covers the
// rounding of both sides (the level already carries the margin M).  Voronoi
// and Laguerre give exactly image_lower(...) <= thr.
template <int KIND, int DIM>
__device__ inline bool lower_passes(const JobConst& C, const TileBox& B, const double* sg, double p, double thr)
{
    double qmin = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double d = fmax(0.0, fmax(B.lo[a] - sg[a], sg[a] - B.hi[a]));
        qmin += d * d;
    }
    if (KIND == KV)
        return qmin <= thr;
    if (KIND == KL)
        return qmin - p <= thr;
    const double r = (thr - p) * C.v;
    return r >= 0.0 && qmin <= (r * r) * (1.0 + 0x1p-40);
}

// True if site c (minimum image sg, parameter p, minimum distance dminc to
// the box) loses to the reference site b on the whole box by more than the
// margin.  Voronoi / Laguerre: key_c - key_b = (e_c - e_b) + 2 x.(g_b - g_c)
// is linear in x, so its minimum over the box is at a corner (e = |g|^2, and
// - w for Laguerre).  Johnson-Mehl: key_c - key_b >= (t_c - t_b) +
// (min distance of c - max distance of b) / v.
template <int KIND, int DIM>
__device__ inline bool beaten_by(const JobConst& C, const TileBox& B, const double* sg, double p, double dminc,
                                 const double* gb, double eb, double tb, double dbmax)
{
    if (KIND == KV || KIND == KL) {
        double ec = 0.0, lin = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            ec += sg[a] * sg[a];
            const double al = gb[a] - sg[a];
            lin += fmin(al * B.lo[a], al * B.hi[a]);
        }
        if (KIND == KL)
            ec -= p;
        return (ec - eb) + 2.0 * lin > C.M;
    }
    return (p - tb) + (dminc - dbmax) * C.rv > C.M;
}

// Every bound of the tile list entry through the site's minimum image sg
// (same outputs as box_bounds for a site whose wrap codes are uniform).
template <int KIND, int DIM>
__device__ inline void image_bounds(const JobConst& C, const TileBox& B, const double* sg, double p, double& lb,
                                    double& ub, double& dmn, double& dmx, double4& g)
{
    double qmin = 0.0, qmax = 0.0, e = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double dmin = fmax(0.0, fmax(B.lo[a] - sg[a], sg[a] - B.hi[a]));
        const double dmax = fmax(fabs(sg[a] - B.lo[a]), fabs(sg[a] - B.hi[a]));
        e += sg[a] * sg[a];
        qmin += dmin * dmin;
        qmax += dmax * dmax;
    }
    if (KIND == KV) {
        lb = qmin;
        ub = qmax;
        dmn = dmx = 0.0;
    } else if (KIND == KL) {
        lb = qmin - p;
        ub = qmax - p;
        e -= p;
        dmn = dmx = 0.0;
    } else {
        dmn = sqrt(qmin);
        dmx = sqrt(qmax);
        lb = p + dmn * C.rv;
        ub = p + dmx * C.rv;
    }
    g = make_double4(sg[0], DIM > 1 ? sg[1] : 0.0, DIM > 2 ? sg[2] : 0.0, e);
}

// Distance a face of the visited bin box must keep from the box of voxel
// centres so that every site beyond it provably loses (key > UB + margin).
template <int KIND>
__device__ inline double needed_reach(const JobConst& C, double UB)
{
    const double t = UB + C.M;
    if (KIND == KV)
        return sqrt(fmax(t, 0.0));
    if (KIND == KL)
        return sqrt(fmax(t + C.pmax, 0.0));
    return fmax(t - C.pmin, 0.0) * C.v;
}

template <int KIND>
__device__ inline double outside_lower_bound(const JobConst& C, double G)
{
    if (KIND == KV)
        return G * G;
    if (KIND == KL)
        return G * G - C.pmax;
    return C.pmin + G * C.rv;
}

// Whether a site whose squared gap to the region's box of voxel centres is g2
// (parameter p) can still have a key <= cut somewhere in the region: Voronoi
// g2 <= cut, Laguerre g2 - w <= cut, Johnson-Mehl t + sqrt(g2) / v <= cut,
// tested on squares with a relative 2^-40 widening (the cut carries the
// margin M).
template <int KIND>
__device__ inline bool may_win_region(const JobConst& C, double g2, double p, double cut)
{
    if (KIND == KV)
        return g2 <= cut;
    if (KIND == KL)
        return g2 - p <= cut;
    const double r = (cut - p) * C.v;
    return r >= 0.0 && g2 <= (r * r) * (1.0 + 0x1p-40);
}

template <typename T>
__device__ inline T sel3(int a, T v0, T v1, T v2)
{
    return a == 0 ? v0 : (a == 1 ? v1 : v2);
}

// Gap between voxel-centre coordinate c (the low / high end of a box) and the
// low face of bin blo / the high face of bin bhi on an axis of length La with
// bins of side bsa (+inf where no site can lie beyond the face).
__device__ inline double face_gap_low(double c, int blo, double bsa, double La, bool periodic)
{
    if (!periodic && blo <= 0)
        return __builtin_inf();
    return c - ((double)blo * bsa + La * 0x1p-30);
}

__device__ inline double face_gap_high(double c, int bhi, int nb, double bsa, double La, bool periodic)
{
    if (!periodic && bhi >= nb - 1)
        return __builtin_inf();
    return ((double)(bhi + 1) * bsa - La * 0x1p-30) - c;
}

// Gap between the box of voxel centres and the low / high face of the bin
// box [blo, bhi] along axis a (+inf where no site can lie beyond the face).
__device__ inline double gap_low(const JobDev& J, const TileBox& B, int a, int blo, bool periodic)
{
    return face_gap_low(B.lo[a], blo, J.bs[a], J.L[a], periodic);
}

__device__ inline double gap_high(const JobDev& J, const TileBox& B, int a, int bhi, bool periodic)
{
    return face_gap_high(B.hi[a], bhi, J.nb[a], J.bs[a], J.L[a], periodic);
}

// Where the site records of a list live: in the list itself (IND false,
// entry k at base[k]) or in the region list (IND true, entry k at
// base[cm[k].y >> 8]).
template <bool IND>
__device__ inline double4 site_at(const double4* base, int k, int flags)
{
    return IND ? base[flags >> 8] : base[k];
}

// True if the listed site e loses to some other listed site on the whole box.
// Voronoi and Laguerre: key_c - key_t = (e_c - e_t) + 2 x.(image_t - image_c),
// linear in x, so its minimum over the box is at a corner.  Johnson-Mehl:
// t_c + d_c/v - (t_t + d_t/v) >= (t_c - t_t) + lbd / v with lbd a lower bound
// of d_c - d_t over the box, from d_c - d_t = (q_c - q_t) / (d_c + d_t).
template <int KIND, int DIM, bool IND>
__device__ inline bool dominated(const double4* base, const double4* cg, const int2* cm, const double2* cq, int e,
                                 unsigned long long refs, const JobConst& C, const TileBox& B)
{
    const double4 gc = cg[e];
    const double tc = KIND == KJM || KIND == KJD ? site_at<IND>(base, e, cm[e].y).w : 0.0;
    const double2 mq = cq[e];
    const bool cgen = (cm[e].y & FL_GENERIC) != 0;
    const double gcv[3] = {gc.x, gc.y, gc.z};
    bool dom = false;
    while (refs) {
        const int t = __ffsll((unsigned long long)refs) - 1;
        refs &= refs - 1;
        const double4 go = cg[t];
        const bool ogen = (cm[t].y & FL_GENERIC) != 0;
        double Dq = 0.0;
        if (!cgen && !ogen) {
            const double gov[3] = {go.x, go.y, go.z};
            double lin = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const double al = gov[a] - gcv[a];
                lin += fmin(al * B.lo[a], al * B.hi[a]);
            }
            Dq = (gc.w - go.w) + 2.0 * lin;
        }
        if (KIND == KV || KIND == KL) {
            dom = dom || (t != e && !cgen && !ogen && Dq > C.M);
        } else {
            // (t_c - t_t) + lbd / v > M with lbd the larger of the two lower
            // bounds of d_c - d_t; the quotient bound Dq / den is tested as
            // Dq / v > (M - (t_c - t_t)) den (den > 0), without a division.
            const double2 oq = cq[t];
            const double dt = tc - site_at<IND>(base, t, cm[t].y).w;
            bool beat = dt + (mq.x - oq.y) * C.rv > C.M;
            if (!cgen && !ogen) {
                const double den = Dq > 0.0 ? mq.y + oq.y : mq.x + oq.x;
                if (den >= C.sqrtL2 * 0x1p-10)
                    beat = beat || Dq * C.rv > (C.M - dt) * den;
            }
            dom = dom || (t != e && beat);
        }
    }
    return dom;
}

// 32-bit ranking key of an upper bound: the high word of the order-preserving
// integer image of the double, with the list position in the low 6 bits
// (distinct keys; close upper bounds may rank in either order, which only
// changes the choice of dominance references).
__device__ inline unsigned ub_key(double u, int pos)
{
    const unsigned hw = (unsigned)((unsigned long long)__double_as_longlong(u) >> 32);
    return (((hw >> 31) ? ~hw : (hw | 0x80000000u)) & ~63u) | (unsigned)pos;
}

// Drops dominated entries of a wavefront's list (one entry per lane, nc <= 64),
// then sorts the rest by site index.  Each entry is tested against the
// r_dom(KIND) entries with the smallest upper bounds (the sites nearest the tile, which
// beat far sites on the whole tile); a dropped entry is always beaten by a
// listed site, so the winner of every voxel stays.  Returns the new count.
// IND false: the list holds the site records (cs, permuted with the list);
// IND true: they stay in the region list `base` (cs unused).
template <int KIND, int DIM, bool IND>
__device__ inline int prune_and_sort(const double4* base, double4* cs, double4* cg, int2* cm, double2* cq,
                                     unsigned* ck, int nc, int lane, const JobConst& C, const TileBox& B)
{
    static_assert(CAP_S == WAVE && CAP_F == WAVE, "one list entry per lane");
    const bool mine = lane < nc;
    bool keep = mine;
    if (nc > 1) {
        // Rank of this entry by upper bound through the keys of ub_key (the
        // caller stored them for entries below nc).
        if (!mine)
            ck[lane] = 0xffffffffu;
        wave_sync();
        const unsigned key = mine ? ck[lane] : 0xffffffffu;
        int ru = 0;
        for (int t = 0; t < nc; t += 4) {
            const uint4 k4 = *(const uint4*)(ck + t);
            ru += (int)(k4.x < key) + (int)(k4.y < key) + (int)(k4.z < key) + (int)(k4.w < key);
        }
        const unsigned long long refs = __ballot(mine && ru < r_dom(KIND));
        keep = !dominated<KIND, DIM, IND>(base, cg, cm, cq, mine ? lane : 0, refs, C, B) && mine;
    }
    double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
    int2 m = make_int2(0, 0);
    if (mine) {
        if (!IND)
            s = cs[lane];
        m = cm[lane];
    }
    const int n = __popcll(__ballot(keep));
    // rank among the kept entries by site index (indices are distinct and
    // below 2^31; dropped entries carry the largest key)
    const unsigned idx = (unsigned)m.x;
    wave_sync();
    ck[lane] = keep ? idx : 0xffffffffu;
    wave_sync();
    int rank = 0;
    for (int t = 0; t < nc; t += 4) {
        const uint4 k4 = *(const uint4*)(ck + t);
        rank += (int)(k4.x < idx) + (int)(k4.y < idx) + (int)(k4.z < idx) + (int)(k4.w < idx);
    }
    wave_sync();
    if (keep) {
        if (!IND)
            cs[rank] = s;
        cm[rank] = m;
    }
    wave_sync();
    return n;
}

// Exact keys of the listed sites (ascending index) at the lane's ROWS runs of
// RUN voxels (row r at y = yv[r]).  The x terms d0*d0 are shared by the rows;
// the sum keeps the grouping d0*d0 + (d1*d1 + d2*d2).
template <int KIND, int DIM, int RUN, int ROWS, bool IND>
__device__ inline void evaluate(const double4* base, const int2* cm, int nc, bool lex, const JobDev& J,
                                const JobConst& C, bool periodic, const double* xr, const double* yv, double zv,
                                double* best, int* lab)
{
    for (int k = 0; k < nc; ++k) {
        const int2 m = cm[k];
        // the list entry is the same for every lane: keep index and flags in
        // scalar registers so that the branches below are scalar
        const int idx = __builtin_amdgcn_readfirstlane(m.x), f = __builtin_amdgcn_readfirstlane(m.y);
        const int fl = f & 0xff;
        const double4 s = site_at<IND>(base, k, f);
        double c[ROWS];
        double dx2[RUN];
        if (fl == 0) {
            const double dz = (DIM == 3) ? s.z - zv : 0.0;
            const double dz2 = dz * dz;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const double dy = s.y - yv[r];
                c[r] = (DIM == 3) ? dy * dy + dz2 : dy * dy;
            }
#pragma unroll
            for (int q = 0; q < RUN; ++q) {
                const double dx = s.x - xr[q];
                dx2[q] = dx * dx;
            }
        } else if (!(fl & FL_GENERIC)) {
            const double dz = (DIM == 3) ? (s.z - zv) + code_off((fl >> 4) & 3, J.L[2]) : 0.0;
            const double dz2 = dz * dz;
            const double oy = code_off((fl >> 2) & 3, J.L[1]);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const double dy = (s.y - yv[r]) + oy;
                c[r] = (DIM == 3) ? dy * dy + dz2 : dy * dy;
            }
            const double ox = code_off(fl & 3, J.L[0]);
#pragma unroll
            for (int q = 0; q < RUN; ++q) {
                const double dx = (s.x - xr[q]) + ox;
                dx2[q] = dx * dx;
            }
        } else {
            const double dz = (DIM == 3) ? (periodic ? min_image(s.z - zv, J.H[2], J.L[2]) : s.z - zv) : 0.0;
            const double dz2 = dz * dz;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const double dy = periodic ? min_image(s.y - yv[r], J.H[1], J.L[1]) : s.y - yv[r];
                c[r] = (DIM == 3) ? dy * dy + dz2 : dy * dy;
            }
#pragma unroll
            for (int q = 0; q < RUN; ++q) {
                const double dx = periodic ? min_image(s.x - xr[q], J.H[0], J.L[0]) : s.x - xr[q];
                dx2[q] = dx * dx;
            }
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            if (!lex) {
#pragma unroll
                for (int q = 0; q < RUN; ++q) {
                    const double key = dist_key<KIND>(dx2[q] + c[r], s.w, C.v, C.rv);
                    lab[r * RUN + q] = key < best[r * RUN + q] ? idx : lab[r * RUN + q];
                    best[r * RUN + q] = fmin(best[r * RUN + q], key);
                }
            } else {
#pragma unroll
                for (int q = 0; q < RUN; ++q) {
                    const double key = dist_key<KIND>(dx2[q] + c[r], s.w, C.v, C.rv);
                    const bool lt = key < best[r * RUN + q] || (key == best[r * RUN + q] && idx < lab[r * RUN + q]);
                    lab[r * RUN + q] = lt ? idx : lab[r * RUN + q];
                    best[r * RUN + q] = fmin(best[r * RUN + q], key);
                }
            }
        }
    }
}

// Writes the evaluation records of the nc sorted list entries (cm, sites in
// the region list `base`) for a tile whose lanes share the x positions xr.
// The records overlay the list arrays, so every lane reads its entry first.
template <int KIND, int DIM>
__device__ inline void write_records(TileLds& S, const double4* base, int nc, int lane, const JobDev& J,
                                     bool periodic, const double* xr)
{
    int2 m = make_int2(0, 0);
    double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
    if (lane < nc) {
        m = S.cm[lane];
        s = base[m.y >> 8];
    }
    int fl = m.y & 0xff;
    if (KIND == KJM || KIND == KJD) {
        // A site off the lattice of voxel centres by at least 2^-24 of a
        // voxel on some axis is that far from every voxel centre (images
        // shift by whole periods); with n < 2^20 the lattice coordinate's
        // rounding error stays below 2^-32.
        const double sc[3] = {s.x, s.y, s.z};
        bool off = false, ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double u = sc[a] / J.h[a] - 0.5;
            off = off || fabs(u - rint(u)) > 0x1p-24;
            ok = ok && J.n[a] < (1 << 20) && J.h[a] > 0x1p-200;
        }
        if (off && ok)
            fl |= FL_SQRT_FAST;
    }
    double d2[XRUN];
    if (!(fl & FL_GENERIC)) {
        const double ox = code_off(fl & 3, J.L[0]);
#pragma unroll
        for (int q = 0; q < XRUN; ++q) {
            const double dx = fl == 0 ? s.x - xr[q] : (s.x - xr[q]) + ox;
            d2[q] = dx * dx;
        }
    } else {
#pragma unroll
        for (int q = 0; q < XRUN; ++q) {
            const double dx = periodic ? min_image(s.x - xr[q], J.H[0], J.L[0]) : s.x - xr[q];
            d2[q] = dx * dx;
        }
    }
    wave_sync();
    if (lane < nc) {
        EvalRec* R = reinterpret_cast<EvalRec*>(&S);
        EvalRec& E = R[lane];
#pragma unroll
        for (int q = 0; q < XRUN; ++q)
            E.dx2[q] = d2[q];
        E.y = s.y;
        E.z = s.z;
        E.p = s.w;
        E.idx = m.x;
        E.flags = fl;
    }
    wave_sync();
}

// evaluate() over evaluation records: the x terms come from LDS.
template <int KIND, int DIM, int ROWS>
__device__ inline void evaluate_rec(const TileLds& S, int nc, const JobDev& J, const JobConst& C, bool periodic,
                                    const double* yv, double zv, double* best, int* lab)
{
    const EvalRec* R = reinterpret_cast<const EvalRec*>(&S);
    for (int k = 0; k < nc; ++k) {
        const EvalRec& E = R[k];
        const int idx = __builtin_amdgcn_readfirstlane(E.idx), fl = __builtin_amdgcn_readfirstlane(E.flags);
        double dx2[XRUN];
#pragma unroll
        for (int q = 0; q < XRUN; ++q)
            dx2[q] = E.dx2[q];
        const double sy = E.y, sz = E.z, sp = E.p;
        double c[ROWS];
        if ((fl & (FL_GENERIC | 0x3c)) == 0) {  // no wrap in y and z
            const double dz = (DIM == 3) ? sz - zv : 0.0;
            const double dz2 = dz * dz;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const double dy = sy - yv[r];
                c[r] = (DIM == 3) ? dy * dy + dz2 : dy * dy;
            }
        } else if (!(fl & FL_GENERIC)) {
            const double dz = (DIM == 3) ? (sz - zv) + code_off((fl >> 4) & 3, J.L[2]) : 0.0;
            const double dz2 = dz * dz;
            const double oy = code_off((fl >> 2) & 3, J.L[1]);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const double dy = (sy - yv[r]) + oy;
                c[r] = (DIM == 3) ? dy * dy + dz2 : dy * dy;
            }
        } else {
            const double dz = (DIM == 3) ? (periodic ? min_image(sz - zv, J.H[2], J.L[2]) : sz - zv) : 0.0;
            const double dz2 = dz * dz;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const double dy = periodic ? min_image(sy - yv[r], J.H[1], J.L[1]) : sy - yv[r];
                c[r] = (DIM == 3) ? dy * dy + dz2 : dy * dy;
            }
        }
        if ((KIND == KJM || KIND == KJD) && (fl & FL_SQRT_FAST)) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
#pragma unroll
                for (int q = 0; q < XRUN; ++q) {
                    const double key = dist_key_fast<KIND>(dx2[q] + c[r], sp, C.v, C.rv);
                    lab[r * XRUN + q] = key < best[r * XRUN + q] ? idx : lab[r * XRUN + q];
                    best[r * XRUN + q] = fmin(best[r * XRUN + q], key);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
#pragma unroll
                for (int q = 0; q < XRUN; ++q) {
                    const double key = dist_key<KIND>(dx2[q] + c[r], sp, C.v, C.rv);
                    lab[r * XRUN + q] = key < best[r * XRUN + q] ? idx : lab[r * XRUN + q];
                    best[r * XRUN + q] = fmin(best[r * XRUN + q], key);
                }
            }
        }
    }
}

template <int RUN, int ROWS>
__device__ inline void store_runs(const JobDev& J, int mi, int mj, int mk, bool bad, int* lab)
{
    if (mk >= J.n[2] || mi >= J.n[0])
        return;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        if (mj + r >= J.n[1])
            break;
        int32_t* out = J.labels + (int64_t)mi + (int64_t)J.n[0] * ((int64_t)(mj + r) + (int64_t)J.n[1] * mk);
        int* l = lab + r * RUN;
        if (bad) {
#pragma unroll
            for (int q = 0; q < RUN; ++q)
                l[q] = -1;
        }
        if (mi + RUN <= J.n[0] && ((uintptr_t)out & 15) == 0 && RUN % 4 == 0) {
#pragma unroll
            for (int q = 0; q < RUN; q += 4)
                *(int4*)(out + q) = make_int4(l[q], l[q + 1], l[q + 2], l[q + 3]);
        } else {
#pragma unroll
            for (int q = 0; q < RUN; ++q)
                if (mi + q < J.n[0])
                    out[q] = l[q];
        }
    }
}

// The winning keys of the lane's runs (the distance image), same layout as
// the labels; NaN for a job with bad input.
template <int RUN, int ROWS>
__device__ inline void store_keys(const JobDev& J, int mi, int mj, int mk, bool bad, const double* best)
{
    if (mk >= J.n[2] || mi >= J.n[0])
        return;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        if (mj + r >= J.n[1])
            break;
        double* out = J.keys + (int64_t)mi + (int64_t)J.n[0] * ((int64_t)(mj + r) + (int64_t)J.n[1] * mk);
        double k[RUN];
#pragma unroll
        for (int q = 0; q < RUN; ++q)
            k[q] = bad ? __builtin_nan("") : best[r * RUN + q];
        if (mi + RUN <= J.n[0] && ((uintptr_t)out & 15) == 0 && RUN % 2 == 0) {
#pragma unroll
            for (int q = 0; q < RUN; q += 2)
                *(double2*)(out + q) = make_double2(k[q], k[q + 1]);
        } else {
#pragma unroll
            for (int q = 0; q < RUN; ++q)
                if (mi + q < J.n[0])
                    out[q] = k[q];
        }
    }
}

// ------------------------------------------------ fallback: one tile alone

// Walks the bins around one tile shell by shell, keeps the sites that can
// win somewhere in the tile and evaluates them in batches of at most CAP_F
// (the first batch with a strict '<' in index order, later ones with the
// lexicographic (key, index) order).  Used when a region's sites overflow LDS.
template <int KIND, int DIM, int RUN, int LX, int LY, int LZ, int ROWS>
__device__ void fallback_tile(const JobDev& J, const JobConst& C, const int* v0, FallbackLds& S, int lane,
                              double* xr, const double* yv, double zv, double* best, int* lab)
{
    constexpr int TX = RUN * LX, TY = LY * ROWS, TZ = (DIM == 3) ? LZ : 1;
    const bool periodic = J.bc != 0;
    const int ve[3] = {min(v0[0] + TX, J.n[0]) - 1, min(v0[1] + TY, J.n[1]) - 1, min(v0[2] + TZ, J.n[2]) - 1};
    const TileBox B = make_box<DIM>(J, v0, ve);
    int blo[3], bhi[3], olo[3], ohi[3];
    for (int a = 0; a < 3; ++a) {
        if (a < DIM) {
            const int l = (int)(B.lo[a] * J.inv_bs[a]), h = (int)(B.hi[a] * J.inv_bs[a]);
            blo[a] = max(0, min(l, J.nb[a] - 1));
            bhi[a] = max(blo[a], min(h, J.nb[a] - 1));
        } else {
            blo[a] = bhi[a] = 0;
        }
        olo[a] = 1;
        ohi[a] = 0;
    }
    int nbx = bhi[0] - blo[0] + 1, nby = bhi[1] - blo[1] + 1, nbz = bhi[2] - blo[2] + 1;
    int64_t sh_total = (int64_t)nbx * nby * nbz, sh_pos = 0;
    int ch_T = 0, ch_off = 0;
    bool ch_live = false;
    double UB = __builtin_inf();
    int nc = 0;
    bool lex = false, done = false;
    for (;;) {
        bool flush = false;
        while (!done && !flush) {
            if (!ch_live) {
                if (sh_pos >= sh_total) {
                    bool complete = true;
                    double G = __builtin_inf();
                    for (int a = 0; a < DIM; ++a) {
                        const bool full = periodic ? (bhi[a] - blo[a] + 1 >= J.nb[a])
                                                   : (blo[a] == 0 && bhi[a] == J.nb[a] - 1);
                        if (full)
                            continue;
                        complete = false;
                        G = fmin(G, fmin(gap_low(J, B, a, blo[a], periodic), gap_high(J, B, a, bhi[a], periodic)));
                    }
                    if (complete || outside_lower_bound<KIND>(C, fmax(G, 0.0)) > UB + C.M) {
                        done = true;
                        break;
                    }
                    for (int a = 0; a < DIM; ++a) {
                        olo[a] = blo[a];
                        ohi[a] = bhi[a];
                        if (periodic) {
                            if (bhi[a] - blo[a] + 1 < J.nb[a]) {
                                blo[a] -= 1;
                                bhi[a] += 1;
                                if (bhi[a] - blo[a] + 1 > J.nb[a])
                                    bhi[a] = blo[a] + J.nb[a] - 1;
                            }
                        } else {
                            blo[a] = max(blo[a] - 1, 0);
                            bhi[a] = min(bhi[a] + 1, J.nb[a] - 1);
                        }
                    }
                    if (DIM == 2)
                        olo[2] = ohi[2] = 0;
                    nbx = bhi[0] - blo[0] + 1;
                    nby = bhi[1] - blo[1] + 1;
                    nbz = bhi[2] - blo[2] + 1;
                    sh_total = (int64_t)nbx * nby * nbz;
                    sh_pos = 0;
                    continue;
                }
                const int64_t e = sh_pos + lane;
                int cnt = 0, src = 0;
                if (e < sh_total) {
                    const int ex = (int)(e % nbx);
                    const int64_t e2 = e / nbx;
                    const int ey = (int)(e2 % nby), ez = (int)(e2 / nby);
                    const int bx = blo[0] + ex, by = blo[1] + ey, bz = blo[2] + ez;
                    const bool old = bx >= olo[0] && bx <= ohi[0] && by >= olo[1] && by <= ohi[1] && bz >= olo[2] &&
                                     bz <= ohi[2];
                    if (!old) {
                        int wx = bx, wy = by, wz = bz;
                        if (periodic) {
                            wx = ((wx % J.nb[0]) + J.nb[0]) % J.nb[0];
                            wy = ((wy % J.nb[1]) + J.nb[1]) % J.nb[1];
                            wz = ((wz % J.nb[2]) + J.nb[2]) % J.nb[2];
                        }
                        const int lin = wx + J.nb[0] * (wy + J.nb[1] * wz);
                        src = J.bin_start[lin];
                        cnt = J.bin_count[lin];
                    }
                }
                const int inc = wave_inclusive_add(cnt, lane);
                S.bcnt[lane] = inc;
                S.bsrc[lane] = src;
                ch_T = __shfl(inc, WAVE - 1);
                ch_off = 0;
                ch_live = ch_T > 0;
                sh_pos += WAVE;
                wave_sync();
                continue;
            }
            const int p = ch_off + lane;
            const bool valid = p < ch_T;
            double4 s = make_double4(0.0, 0.0, 0.0, 0.0), g = s;
            int sid = 0, flags = 0;
            double lb = __builtin_inf(), ub = __builtin_inf(), dmn = 0.0, dmx = 0.0;
            if (valid) {
                int lo = 0, hi = WAVE - 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (S.bcnt[mid] > p)
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                const int excl = lo == 0 ? 0 : S.bcnt[lo - 1];
                const int pos = S.bsrc[lo] + (p - excl);
                s = J.sites[pos];
                sid = J.sidx[pos];
                box_bounds<KIND, DIM>(J, C, B, periodic, s, flags, lb, ub, dmn, dmx, g);
            }
            UB = fmin(UB, wave_min(ub));
            const bool keep = valid && lb <= UB + C.M;
            const unsigned long long km = __ballot(keep);
            if (keep) {
                const int slot = nc + __popcll(km & lanes_below(lane));
                S.cs[slot] = s;
                S.cg[slot] = g;
                S.cb[slot] = make_double2(lb, ub);
                S.cq[slot] = make_double2(dmn, dmx);
                S.cm[slot] = make_int2(sid, flags);
            }
            nc += __popcll(km);
            ch_off += WAVE;
            if (ch_off >= ch_T)
                ch_live = false;
            wave_sync();
            if (nc > CAP_F - WAVE)
                flush = true;
        }
        if (nc > 0) {
            // keep the entries under the current UB, then prune, sort, evaluate
            const double thr = UB + C.M;
            double4 s = make_double4(0.0, 0.0, 0.0, 0.0), g = s;
            double2 q = make_double2(0.0, 0.0);
            double u = 0.0;
            int2 m = make_int2(0, 0);
            bool keep = false;
            if (lane < nc) {
                s = S.cs[lane];
                g = S.cg[lane];
                const double2 b = S.cb[lane];
                u = b.y;
                q = S.cq[lane];
                m = S.cm[lane];
                keep = b.x <= thr;
            }
            const unsigned long long km = __ballot(keep);
            wave_sync();
            if (keep) {
                const int d = __popcll(km & lanes_below(lane));
                S.cs[d] = s;
                S.cg[d] = g;
                S.ck[d] = ub_key(u, d);
                S.cq[d] = q;
                S.cm[d] = m;
            }
            nc = __popcll(km);
            wave_sync();
            nc = prune_and_sort<KIND, DIM, false>(S.cs, S.cs, S.cg, S.cm, S.cq, S.ck, nc, lane, C, B);
            evaluate<KIND, DIM, RUN, ROWS, false>(S.cs, S.cm, nc, lex, J, C, periodic, xr, yv, zv, best, lab);
            lex = true;
            nc = 0;
            wave_sync();
        }
        if (done)
            break;
    }
}

// ------------------------------------------------------------ one region

struct LaneGeo {
    int t0[3];      // first voxel of the tile
    bool live;      // tile inside the grid
    int mi, mj, mk; // first voxel of the lane's run
};

// Region coordinates of region r (regions are numbered x fastest; fewer
// than 2^31 per job).
__device__ inline void region_coords(const JobDev& J, int64_t r, int& rx, int& ry, int& rz)
{
    const unsigned u = (unsigned)r, n0 = (unsigned)J.nr[0], n1 = (unsigned)J.nr[1];
    const unsigned q = u / n0;
    rx = (int)(u - q * n0);
    rz = (int)(q / n1);
    ry = (int)(q - (unsigned)rz * n1);
}

template <int DIM, int RUN, int LX, int LY, int LZ, int ROWS, int RX, int RY, int RZ>
__device__ inline LaneGeo lane_geometry(const JobDev& J, int64_t r, int w, int lane)
{
    constexpr int TX = RUN * LX, TY = LY * ROWS, TZ = (DIM == 3) ? LZ : 1;
    int rx, ry, rz;
    region_coords(J, r, rx, ry, rz);
    LaneGeo G;
    G.t0[0] = rx * TX * RX + (w % RX) * TX;
    G.t0[1] = ry * TY * RY + ((w / RX) % RY) * TY;
    G.t0[2] = rz * TZ * RZ + (w / (RX * RY)) * TZ;
    G.live = G.t0[0] < J.n[0] && G.t0[1] < J.n[1] && G.t0[2] < J.n[2];
    const int lx = lane % LX, ly = (lane / LX) % LY, lz = lane / (LX * LY);
    G.mi = G.t0[0] + lx * RUN;
    G.mj = G.t0[1] + ly * ROWS;
    G.mk = (DIM == 3) ? G.t0[2] + lz : 0;
    return G;
}

// Region `r` of job J: NW tiles of shape T (tile w of the region is processed
// by wavefront w), RX x RY x RZ tiles.  `unit` numbers the region in the
// launch (job-local, or batch-wide) for the overflow list.
//
// DENSE false (main kernels): a region whose gather overflows the region list
// is queued whole on the overflow list (as -(unit + 1)), a tile whose
// candidate list overflows as unit * NW + w.  DENSE true (overflow kernels):
// a first box too dense for the list starts over from the region's own bins
// and the later rounds load only sites that can still win (every kind); the
// return value tells the wavefront whose tile still overflows (its labels are
// not stored) to label it with the per-tile walk.
template <int KIND, int DIM, int RUN, int LX, int LY, int LZ, int ROWS, int RX, int RY, int RZ, bool DENSE>
__device__ bool label_region(const JobDev& J, int64_t r, int64_t unit, Smem& sm, const int tid)
{
    constexpr int TX = RUN * LX, TY = LY * ROWS, TZ = (DIM == 3) ? LZ : 1;
    static_assert(LX * LY * LZ == WAVE, "64 lanes per tile");
    static_assert(RX * RY * RZ == NW, "one tile per wavefront");
    const bool periodic = J.bc != 0;
    const int lane = tid & (WAVE - 1), w = tid / WAVE;

    // ---- region and tile geometry
    int rx, ry, rz;
    region_coords(J, r, rx, ry, rz);
    const int r0[3] = {rx * TX * RX, ry * TY * RY, rz * TZ * RZ};
    const int re[3] = {min(r0[0] + TX * RX, J.n[0]) - 1, min(r0[1] + TY * RY, J.n[1]) - 1,
                       min(r0[2] + TZ * RZ, J.n[2]) - 1};
    const TileBox BR = make_box<DIM>(J, r0, re);
    const LaneGeo G = lane_geometry<DIM, RUN, LX, LY, LZ, ROWS, RX, RY, RZ>(J, r, w, lane);
    const int te[3] = {min(G.t0[0] + TX, J.n[0]) - 1, min(G.t0[1] + TY, J.n[1]) - 1,
                       min(G.t0[2] + TZ, J.n[2]) - 1};
    const TileBox BT = make_box<DIM>(J, G.t0, te);

    int lab[ROWS * RUN];
#pragma unroll
    for (int q = 0; q < ROWS * RUN; ++q)
        lab[q] = -1;

    const bool bad = *(volatile int32_t*)J.status != 0;
    bool tile_ovf = false, region_ovf = false;
    if (!bad) {
        const JobConst C = job_const<KIND>(J, DIM);
        RegionLds& R = sm.r.reg;

        // ======== 1. region gather (whole workgroup)
        int blo[3], bhi[3], olo[3], ohi[3], own_lo[3], own_hi[3];
        for (int a = 0; a < 3; ++a) {
            own_lo[a] = own_hi[a] = 0;
            if (a < DIM) {
                const int nb = J.nb[a];
                int l = (int)(BR.lo[a] * J.inv_bs[a]), h = (int)(BR.hi[a] * J.inv_bs[a]);
                l = max(0, min(l, nb - 1));
                h = max(l, min(h, nb - 1));
                own_lo[a] = l;
                own_hi[a] = h;
                // first box: the region's bins and GM more on each side.
                // Johnson-Mehl reaches farther: its gather would almost
                // always need a second round from one.  Laguerre takes the
                // margin its plan gives (two with bins near the mean spacing,
                // one with the large bins of sparse grids, whose first box
                // would otherwise overflow).
                const int GM = (KIND == KJM || KIND == KJD) ? 2 : (KIND == KL ? J.gather_margin : 1);
                if (periodic) {
                    blo[a] = l - GM;
                    bhi[a] = h + GM;
                    if (bhi[a] - blo[a] + 1 >= nb) {
                        blo[a] = l;
                        bhi[a] = l + nb - 1;
                    }
                } else {
                    blo[a] = max(l - GM, 0);
                    bhi[a] = min(h + GM, nb - 1);
                }
            } else {
                blo[a] = bhi[a] = 0;
            }
            olo[a] = 1;
            ohi[a] = 0;
        }
        int nR = 0, nDone = 0;
        bool overflow = false, dense = false, restart = false;
        double skip_cut = __builtin_inf();  // UB + M of the previous round (load test)
        double ubT = __builtin_inf();  // this tile's upper bound (wave-uniform)
        int ubPos = -1;                // region-list position of a site attaining it
        for (int round = 0;; ++round) {
            // load every bin of the box that is not in the previous box
            const int nbx = bhi[0] - blo[0] + 1, nby = bhi[1] - blo[1] + 1, nbz = bhi[2] - blo[2] + 1;
            const int64_t nbox = (int64_t)nbx * nby * nbz;
            if (nbox >= (1 << 30)) {  // beyond the bin decoding's range: leave it to the fallback
                overflow = true;
                break;
            }
            const float rnx = 1.0f / (float)nbx, rnxy = 1.0f / (float)(nbx * nby);
            for (int64_t base = 0; base < nbox; base += NT) {
                const int64_t e = base + tid;
                int cnt = 0, src = 0, code = 0;
                if (e < nbox) {
                    int rxy, ex;
                    const int ez = divmod_small((int)e, nbx * nby, rnxy, rxy);
                    const int ey = divmod_small(rxy, nbx, rnx, ex);
                    const int bx = blo[0] + ex, by = blo[1] + ey, bz = blo[2] + ez;
                    const bool old = bx >= olo[0] && bx <= ohi[0] && by >= olo[1] && by <= ohi[1] && bz >= olo[2] &&
                                     bz <= ohi[2];
                    if (!old) {
                        int wx = bx, wy = by, wz = bz;
                        if (periodic) {
                            wx = wrap_bin(wx, J.nb[0]);
                            wy = wrap_bin(wy, J.nb[1]);
                            wz = wrap_bin(wz, J.nb[2]);
                            // image of the bin's sites: shifted by -L below the
                            // grid (code 1), by +L above it (code 2)
                            code = (bx < 0 ? 1 : (bx >= J.nb[0] ? 2 : 0)) |
                                   ((by < 0 ? 1 : (by >= J.nb[1] ? 2 : 0)) << 2) |
                                   ((bz < 0 ? 1 : (bz >= J.nb[2] ? 2 : 0)) << 4);
                        }
                        const int lin = wx + J.nb[0] * (wy + J.nb[1] * wz);
                        src = J.bin_start[lin];
                        cnt = J.bin_count[lin];
                    }
                }
                int total;
                int off = block_excl_scan(cnt, total, R.wsum, tid);
                // From the second round on, when the round's bins would
                // overflow the list: a site whose own lower bound over the
                // region (from the gap to its nearest periodic image; for
                // Laguerre the gap squared minus its weight, for Johnson-Mehl
                // its time plus the gap over v) exceeds UB + M loses at every
                // voxel, so it is not loaded.  This keeps the list within
                // LDS where sites are dense (clusters), and keeps one heavy
                // Laguerre site, whose weight sets everyone's reach, from
                // overflowing the lists of every region near it.  (The
                // condition is the same for the whole workgroup; bins of more
                // than 64 sites load whole.)
                unsigned long long keep = ~0ull;
                const bool filtered = (DENSE || KIND == KL) && nR + total > CAP_R && skip_cut < __builtin_inf();
                if (filtered) {
                    int nload = cnt;
                    if (cnt > 0 && cnt <= 64) {
                        keep = 0ull;
                        nload = 0;
                        for (int k = 0; k < cnt; ++k) {
                            const double4 sv = J.sites[src + k];
                            const double sc[3] = {sv.x, sv.y, sv.z};
                            double g2 = 0.0;
#pragma unroll
                            for (int a = 0; a < DIM; ++a) {
                                double gap = fmax(BR.lo[a] - sc[a], sc[a] - BR.hi[a]);
                                if (periodic) {
                                    const double lo = sc[a] - J.L[a], hi = sc[a] + J.L[a];
                                    gap = fmin(gap, fmin(fmax(BR.lo[a] - lo, lo - BR.hi[a]),
                                                         fmax(BR.lo[a] - hi, hi - BR.hi[a])));
                                }
                                g2 += gap > 0.0 ? gap * gap : 0.0;
                            }
                            if (may_win_region<KIND>(C, g2, sv.w, skip_cut)) {
                                keep |= 1ull << k;
                                ++nload;
                            }
                        }
                    }
                    off = block_excl_scan(nload, total, R.wsum, tid);
                }
                if (nR + total > CAP_R) {
                    // (Overflow kernels) a first box too dense for the list
                    // starts over from the region's own bins; the rounds
                    // after it load through the test above.
                    if (DENSE && round == 0 && !dense)
                        restart = true;
                    else
                        overflow = true;
                    break;
                }
                // Each bin first writes the sorted position and wrap code of
                // its sites into their list slots (LDS only); then one thread
                // per slot loads its site, so that every global load of the
                // round is in flight at once instead of one bin's sites
                // following each other.
                if (!filtered) {
                    for (int k = 0; k < cnt; ++k) {
                        R.ri[nR + off + k] = src + k;
                        R.rf[nR + off + k] = code;
                    }
                } else {
                    for (int k = 0, d = 0; k < cnt; ++k) {
                        // bins of more than 64 sites load whole (keep has one
                        // bit per site of the smaller bins only)
                        if (k < 64 && !((keep >> k) & 1ull))
                            continue;
                        R.ri[nR + off + d] = src + k;
                        R.rf[nR + off + d] = code;
                        ++d;
                    }
                }
                __syncthreads();
                for (int p = tid; p < total; p += NT) {
                    const int sp = R.ri[nR + p];
                    R.rs[nR + p] = J.sites[sp];
                    R.ri[nR + p] = J.sidx[sp];
                }
                nR += total;
            }
            if (DENSE && restart) {
                restart = false;
                dense = true;
                for (int a = 0; a < 3; ++a) {
                    blo[a] = own_lo[a];
                    bhi[a] = own_hi[a];
                    olo[a] = 1;
                    ohi[a] = 0;
                }
                nR = 0;
                round = -1;
                __syncthreads();
                continue;
            }
            if (overflow)
                break;
            __syncthreads();
            // Each tile's upper bound from the sites added in this round; the
            // region's stopping level is the largest of them (every voxel of
            // the region then has a winning key below it).
            bool wrapped = false;
            if (periodic)
                for (int a = 0; a < DIM; ++a)
                    wrapped = wrapped || blo[a] < 0 || bhi[a] >= J.nb[a];
            double ubm = __builtin_inf();
            int posm = -1;
            for (int e = nDone + lane; e < nR; e += WAVE) {
                const double4 sv = R.rs[e];
                double sg[3];
                site_image<DIM>(J, sv, R.rf[e], wrapped, sg);
                const double u = image_upper<KIND, DIM>(C, BT, sg, sv.w);
                posm = u < ubm ? e : posm;
                ubm = fmin(ubm, u);
            }
            const double rmin = wave_min(ubm);
            if (rmin < ubT) {
                ubT = rmin;
                ubPos = __builtin_amdgcn_readlane(posm, __ffsll((unsigned long long)__ballot(ubm == rmin)) - 1);
            }
            nDone = nR;
            const double UB = block_max(G.live ? ubT : -__builtin_inf(), R.wred, tid);
            skip_cut = UB + C.M;
            // move the faces that are too close
            const double reach = needed_reach<KIND>(C, UB);
            const double need = reach + reach * 0x1p-20 + 1e-300;
            // One lane per face of the bin box (lane 2a: low face of axis a,
            // lane 2a + 1: high face): move it out until the gap between the
            // region's voxel centres and the face exceeds `need`.
            int fnew = 0;
            if (lane < 2 * DIM) {
                const int a = lane >> 1;
                const bool high = (lane & 1) != 0;
                const int nb = sel3(a, J.nb[0], J.nb[1], J.nb[2]);
                const double La = sel3(a, J.L[0], J.L[1], J.L[2]), bsa = sel3(a, J.bs[0], J.bs[1], J.bs[2]);
                const double inv = sel3(a, J.inv_bs[0], J.inv_bs[1], J.inv_bs[2]);
                const double blo_c = sel3(a, BR.lo[0], BR.lo[1], BR.lo[2]), bhi_c = sel3(a, BR.hi[0], BR.hi[1], BR.hi[2]);
                const int lo0 = sel3(a, blo[0], blo[1], blo[2]), hi0 = sel3(a, bhi[0], bhi[1], bhi[2]);
                int res = high ? hi0 : lo0;
                if (!(periodic && hi0 - lo0 + 1 >= nb)) {
                    if (periodic && need >= La) {
                        res = high ? lo0 + nb - 1 : lo0;
                    } else if (!high) {
                        int lo = lo0;
                        if (face_gap_low(blo_c, lo, bsa, La, periodic) <= need) {
                            const int t = (int)fmax(floor((blo_c - need) * inv), -1.0 * nb - 1.0);
                            lo = min(lo - 1, t);
                            if (!periodic)
                                lo = max(lo, 0);
                            while (face_gap_low(blo_c, lo, bsa, La, periodic) <= need && (periodic || lo > 0))
                                --lo;
                        }
                        res = lo;
                    } else {
                        int hi = hi0;
                        if (face_gap_high(bhi_c, hi, nb, bsa, La, periodic) <= need) {
                            const int t = (int)fmin(floor((bhi_c + need) * inv), 2.0 * nb + 1.0);
                            hi = max(hi + 1, t);
                            if (!periodic)
                                hi = min(hi, nb - 1);
                            while (face_gap_high(bhi_c, hi, nb, bsa, La, periodic) <= need &&
                                   (periodic || hi < nb - 1))
                                ++hi;
                        }
                        res = hi;
                    }
                }
                fnew = res;
            }
            bool moved = false;
            int nlo[3], nhi[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nlo[a] = blo[a];
                nhi[a] = bhi[a];
                if (a < DIM) {
                    int lo = __builtin_amdgcn_readlane(fnew, 2 * a), hi = __builtin_amdgcn_readlane(fnew, 2 * a + 1);
                    if (periodic && hi - lo + 1 >= J.nb[a]) {
                        lo = blo[a];
                        hi = blo[a] + J.nb[a] - 1;
                    }
                    moved = moved || lo != blo[a] || hi != bhi[a];
                    nlo[a] = lo;
                    nhi[a] = hi;
                }
            }
            if (!moved)
                break;
            for (int a = 0; a < 3; ++a) {
                olo[a] = blo[a];
                ohi[a] = bhi[a];
                blo[a] = nlo[a];
                bhi[a] = nhi[a];
            }
            if (round > 64) {  // every round grows the box; leave pathological cases to the fallback
                overflow = true;
                break;
            }
        }
        __syncthreads();

        // ======== 2-3. per tile: prune and evaluate (one wavefront)
        // The images the gather assigned by bin are the minimum images for
        // every voxel of the region when, on each periodic axis, the gather
        // box stays within half a period of the region's voxels: the wrap
        // decision d >= L/2 / d < -L/2 on d = s - x is then the same for all
        // of them (the slack covers bin-edge rounding).
        bool img_ok = true, wrapped = false;
        if (periodic) {
            for (int a = 0; a < DIM; ++a)
                wrapped = wrapped || blo[a] < 0 || bhi[a] >= J.nb[a];
            for (int a = 0; a < DIM; ++a) {
                const double ext = fmax((double)(bhi[a] + 1) * J.bs[a] - BR.lo[a], BR.hi[a] - (double)blo[a] * J.bs[a]);
                img_ok = img_ok && ext < J.H[a] - J.L[a] * 0x1p-30;
            }
        }
        tile_ovf = overflow;
        region_ovf = overflow;
        if (!overflow && G.live) {
            TileLds& S = sm.r.tile[w];
            const double thr = ubT + C.M;
            int nc = 0;
            if (img_ok) {
                // Lower-bound test over the whole region list, together with
                // a dominance test against the site attaining the tile's
                // upper bound (the site nearest the tile); then the full
                // bounds of the survivors only.
                double gb[3] = {0.0, 0.0, 0.0}, eb = 0.0, tb = 0.0, dbmax = 0.0;
                if (ubPos >= 0) {
                    const double4 sb = R.rs[ubPos];
                    site_image<DIM>(J, sb, R.rf[ubPos], wrapped, gb);
                    double qb = 0.0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        eb += gb[a] * gb[a];
                        const double dmax = fmax(fabs(gb[a] - BT.lo[a]), fabs(gb[a] - BT.hi[a]));
                        qb += dmax * dmax;
                    }
                    if (KIND == KL)
                        eb -= sb.w;
                    tb = sb.w;
                    if (KIND == KJM || KIND == KJD)
                        dbmax = sqrt(qb);
                }
                // Voronoi and Laguerre, pass 1: the lower-bound test alone over
                // the region list, survivors staged in S.ci; pass 2: full
                // bounds and the reference test of the staged sites, compacted.
                // A tile with more than CAP_S survivors of pass 1, and every
                // Johnson-Mehl tile (whose lower bound alone keeps many more
                // sites), take both tests in one pass instead.
                int nst = 0;
                bool many = KIND == KJM || KIND == KJD;
                for (int ebase = 0; ebase < (many ? 0 : nR); ebase += WAVE) {
                    const int e = ebase + lane;
                    bool keep = false;
                    if (e < nR) {
                        const double4 sv = R.rs[e];
                        double sg[3];
                        site_image<DIM>(J, sv, R.rf[e], wrapped, sg);
                        keep = lower_passes<KIND, DIM>(C, BT, sg, sv.w, thr);
                    }
                    const unsigned long long km = __ballot(keep);
                    if (nst + __popcll(km) > CAP_S) {
                        many = true;
                        break;
                    }
                    if (keep)
                        S.ci[nst + __popcll(km & lanes_below(lane))] = e;
                    nst += __popcll(km);
                }
                if (many) {
                    nst = 0;
                    for (int ebase = 0; ebase < nR; ebase += WAVE) {
                        const int e = ebase + lane;
                        bool keep = false;
                        if (e < nR) {
                            const double4 sv = R.rs[e];
                            double sg[3];
                            site_image<DIM>(J, sv, R.rf[e], wrapped, sg);
                            double dminc;
                            keep = image_lower_d<KIND, DIM>(C, BT, sg, sv.w, dminc) <= thr;
                            if (keep && ubPos >= 0 && e != ubPos)
                                keep = !beaten_by<KIND, DIM>(C, BT, sg, sv.w, dminc, gb, eb, tb, dbmax);
                        }
                        const unsigned long long km = __ballot(keep);
                        if (nst + __popcll(km) > CAP_S) {
                            tile_ovf = true;
                            break;
                        }
                        if (keep)
                            S.ci[nst + __popcll(km & lanes_below(lane))] = e;
                        nst += __popcll(km);
                    }
                }
                wave_sync();
                bool keep = false;
                int e = 0, code = 0;
                double ub = 0.0, dmn = 0.0, dmx = 0.0;
                double4 g = make_double4(0.0, 0.0, 0.0, 0.0);
                if (!tile_ovf && lane < nst) {
                    e = S.ci[lane];
                    const double4 sv = R.rs[e];
                    code = R.rf[e];
                    double sg[3], lb;
                    site_image<DIM>(J, sv, code, wrapped, sg);
                    image_bounds<KIND, DIM>(C, BT, sg, sv.w, lb, ub, dmn, dmx, g);
                    keep = true;
                    if (!many && ubPos >= 0 && e != ubPos)
                        keep = !beaten_by<KIND, DIM>(C, BT, sg, sv.w, dmn, gb, eb, tb, dbmax);
                }
                const unsigned long long km = __ballot(keep);
                wave_sync();  // every staged position is read before ck (over ci) is written
                if (keep) {
                    const int slot = __popcll(km & lanes_below(lane));
                    S.cg[slot] = g;
                    S.cq[slot] = make_double2(dmn, dmx);
                    S.ck[slot] = ub_key(ub, slot);
                    S.cm[slot] = make_int2(R.ri[e], code | (e << 8));
                }
                nc = tile_ovf ? 0 : __popcll(km);
            } else {
                // Images per tile (box_bounds).  The reference test runs for
                // sites whose wrap code is uniform over the tile, against the
                // site attaining the tile's upper bound when its own is too.
                double gb[3] = {0.0, 0.0, 0.0}, eb = 0.0, tb = 0.0, dbmax = 0.0;
                bool ref_ok = false;
                if (ubPos >= 0) {
                    int fb;
                    double lbb, ubb, dmnb;
                    double4 g4;
                    const double4 sb = R.rs[ubPos];
                    box_bounds<KIND, DIM>(J, C, BT, periodic, sb, fb, lbb, ubb, dmnb, dbmax, g4);
                    ref_ok = (fb & FL_GENERIC) == 0;
                    gb[0] = g4.x;
                    gb[1] = g4.y;
                    gb[2] = g4.z;
                    eb = g4.w;
                    tb = sb.w;
                }
                for (int ebase = 0; ebase < nR; ebase += WAVE) {
                    const int e = ebase + lane;
                    int flags = 0;
                    double lb = __builtin_inf(), ub, dmn = 0.0, dmx = 0.0;
                    double4 s = make_double4(0.0, 0.0, 0.0, 0.0), g = s;
                    if (e < nR) {
                        s = R.rs[e];
                        box_bounds<KIND, DIM>(J, C, BT, periodic, s, flags, lb, ub, dmn, dmx, g);
                    }
                    bool keep = e < nR && lb <= thr;
                    if (keep && ref_ok && (flags & FL_GENERIC) == 0 && e != ubPos) {
                        const double sg[3] = {g.x, g.y, g.z};
                        keep = !beaten_by<KIND, DIM>(C, BT, sg, s.w, dmn, gb, eb, tb, dbmax);
                    }
                    const unsigned long long km = __ballot(keep);
                    if (nc + __popcll(km) > CAP_S) {
                        tile_ovf = true;
                        break;
                    }
                    if (keep) {
                        const int slot = nc + __popcll(km & lanes_below(lane));
                        S.cg[slot] = g;
                        S.cq[slot] = make_double2(dmn, dmx);
                        S.ck[slot] = ub_key(ub, slot);
                        S.cm[slot] = make_int2(R.ri[e], flags | (e << 8));
                    }
                    nc += __popcll(km);
                }
            }
            wave_sync();
            if (!tile_ovf) {
                nc = prune_and_sort<KIND, DIM, true>(R.rs, S.cg, S.cg, S.cm, S.cq, S.ck, nc, lane, C, BT);
                // the lane's voxel centres (computed here so that they do not
                // hold registers through the gather)
                double xr[RUN];
#pragma unroll
                for (int q = 0; q < RUN; ++q)
                    xr[q] = ((double)(G.mi + q) + 0.5) * J.h[0];
                double yv[ROWS];
#pragma unroll
                for (int rr = 0; rr < ROWS; ++rr)
                    yv[rr] = ((double)(G.mj + rr) + 0.5) * J.h[1];
                const double zv = (DIM == 3) ? ((double)G.mk + 0.5) * J.h[2] : 0.0;
                double best[ROWS * RUN];
#pragma unroll
                for (int q = 0; q < ROWS * RUN; ++q)
                    best[q] = __builtin_inf();
                if (RUN == XRUN && LX == 1 && nc <= CAP_E) {
                    write_records<KIND, DIM>(S, R.rs, nc, lane, J, periodic, xr);
                    evaluate_rec<KIND, DIM, ROWS>(S, nc, J, C, periodic, yv, zv, best, lab);
                } else {
                    evaluate<KIND, DIM, RUN, ROWS, true>(R.rs, S.cm, nc, false, J, C, periodic, xr, yv, zv, best, lab);
                }
                if (J.keys)
                    store_keys<RUN, ROWS>(J, G.mi, G.mj, G.mk, false, best);
            }
        }
    }
    if (!DENSE && region_ovf) {
        // leave the whole region to the overflow kernel
        if (tid == 0) {
            const int pos = atomicAdd(J.ovf_count, 1);
            J.ovf_list[pos] = (int32_t)(-unit - 1);
        }
    } else if (G.live) {
        if (tile_ovf) {
            if (DENSE) {
                return true;
            } else if (lane == 0) {
                // leave this tile to the overflow kernel
                const int pos = atomicAdd(J.ovf_count, 1);
                J.ovf_list[pos] = (int32_t)(unit * NW + w);
            }
        } else {
            store_runs<RUN, ROWS>(J, G.mi, G.mj, G.mk, bad, lab);
            if (bad && J.keys) {
                double none[ROWS * RUN];
#pragma unroll
                for (int q = 0; q < ROWS * RUN; ++q)
                    none[q] = 0.0;
                store_keys<RUN, ROWS>(J, G.mi, G.mj, G.mk, true, none);
            }
        }
    }
    return false;
}

// One tile of the overflow list, alone (fallback path, one wavefront).
template <int KIND, int DIM, int RUN, int LX, int LY, int LZ, int ROWS, int RX, int RY, int RZ>
__device__ void label_tile_alone(const JobDev& J, int64_t r, int w, FallbackLds& S, int lane)
{
    const LaneGeo G = lane_geometry<DIM, RUN, LX, LY, LZ, ROWS, RX, RY, RZ>(J, r, w, lane);
    if (!G.live)
        return;
    double xr[RUN];
#pragma unroll
    for (int q = 0; q < RUN; ++q)
        xr[q] = ((double)(G.mi + q) + 0.5) * J.h[0];
    double yv[ROWS];
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr)
        yv[rr] = ((double)(G.mj + rr) + 0.5) * J.h[1];
    const double zv = (DIM == 3) ? ((double)G.mk + 0.5) * J.h[2] : 0.0;
    double best[ROWS * RUN];
    int lab[ROWS * RUN];
#pragma unroll
    for (int q = 0; q < ROWS * RUN; ++q) {
        best[q] = __builtin_inf();
        lab[q] = -1;
    }
    const bool bad = *(volatile int32_t*)J.status != 0;
    if (!bad) {
        const JobConst C = job_const<KIND>(J, DIM);
        fallback_tile<KIND, DIM, RUN, LX, LY, LZ, ROWS>(J, C, G.t0, S, lane, xr, yv, zv, best, lab);
    }
    store_runs<RUN, ROWS>(J, G.mi, G.mj, G.mk, bad, lab);
    if (J.keys)
        store_keys<RUN, ROWS>(J, G.mi, G.mj, G.mk, bad, best);
}

// Consecutive regions go to one XCD: workgroups are dispatched to the eight
// XCDs round-robin, so workgroup b runs on XCD b % 8; give each XCD a
// contiguous range so that neighbouring regions share its L2.
__device__ inline int64_t xcd_unit(int64_t b, int64_t G)
{
    const int64_t x = b & 7, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

template <int KIND, int DIM, int CFG>
__device__ inline void region_cfg(const JobDev& J, int64_t r, int64_t unit, Smem& sm, int tid)
{
    constexpr TileShape T = (DIM == 3) ? kShape3[CFG] : kShape2[CFG];
    label_region<KIND, DIM, T.run, T.lx, T.ly, T.lz, T.rows, T.rx, T.ry, T.rz, false>(J, r, unit, sm, tid);
}

// A region the main kernel queued whole (its gather overflowed), with the
// dense-capable gather (overflow kernels); true for a wavefront whose tile is
// left to the per-tile walk.
template <int KIND, int DIM, int CFG>
__device__ inline bool region_dense_cfg(const JobDev& J, int64_t r, Smem& sm, int tid)
{
    constexpr TileShape T = (DIM == 3) ? kShape3[CFG] : kShape2[CFG];
    return label_region<KIND, DIM, T.run, T.lx, T.ly, T.lz, T.rows, T.rx, T.ry, T.rz, true>(J, r, r, sm, tid);
}

template <int KIND, int DIM, int CFG>
__device__ inline void alone_cfg(const JobDev& J, int64_t r, int w, FallbackLds& S, int lane)
{
    constexpr TileShape T = (DIM == 3) ? kShape3[CFG] : kShape2[CFG];
    label_tile_alone<KIND, DIM, T.run, T.lx, T.ly, T.lz, T.rows, T.rx, T.ry, T.rz>(J, r, w, S, lane);
}

constexpr int kFallbackGrid = 256;  // workgroups of the overflow kernels (each holds 68 KB of LDS)

}  // namespace
}  // namespace vt
