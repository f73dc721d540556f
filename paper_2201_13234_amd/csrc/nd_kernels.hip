// nd_kernels.hip -- the general path: diagrams in any dimension d = 1 .. 6
// (the paper states the method for any dimension, Sec. 3 problem statement),
// with anisotropic voxels and the same keys as the 2D/3D path:
//     Voronoi q,  Laguerre q - w_s,  Johnson-Mehl t_s + sqrt(q) / v,
// q = d0*d0 + T, T = d1*d1, then T + d2*d2, ... over the remaining axes (the
// 2D and 3D forms are its first cases), each operation rounded once.
//
// Periodic boundaries come in two forms (App. A):
//   - orthogonal periods L_a: minimum-image differences (eq. dL), sites
//     brought into the cell first;
//   - general period vectors L_i (eq. L-distance_def, "lattice"): voxel k is
//     centred at x_a = sum_i (k_i + 1/2) (L_ia / n_i), and q is the minimum
//     over integer translations k of the folded sum of d_a^2 with
//     d_a = (s_a - x_a) + (k_0 L_0a + k_1 L_1a + ...).
//
// Binning: a counting sort into a uniform d-dimensional bin grid (in
// fractional coordinates for general periods).
//
// Labelling: one workgroup of 256 threads per tile of at most 256 voxels
// (powers of two per axis), one voxel per thread (two along axis 0 on large
// grids with orthogonal periods in 2 to 4 axes).
//   1. The box of visited bins around the tile grows (face by face, or by
//      whole rings for general periods) until the sites beyond it provably
//      lose: UB = the smallest upper bound of a visited site's key over the
//      tile's voxel centres, and the sites beyond a face are at least its
//      `gap` away, so their keys exceed gap^2 (Voronoi), gap^2 - max w
//      (Laguerre), min t + gap / v (Johnson-Mehl).  With orthogonal periods
//      each round lists its new bins' sites in LDS, one site per thread, and
//      stages the sites whose lower bound is within the current UB + M.
//   2. The visited sites whose lower bound over the tile is <= UB + M are
//      kept in LDS (for general periods, staged after the search with the
//      box of translations that can bring them within reach).  Voronoi and
//      Laguerre with orthogonal periods drop those that the site attaining UB
//      beats on the whole tile (linear key difference).  Every thread takes
//      the lexicographic minimum of (key, site index) over the rest: the
//      brute-force result with ties to the lowest index, whatever the order
//      of the candidates.  With orthogonal periods the per-axis squared
//      differences come from a table formed once per tile.
// M = 2^-36 of the key scale, far above the rounding error of any bound or
// key, so a dropped site's (or translation's) computed key is strictly
// above the winner's.
#include "nd_internal.h"

namespace vt {

namespace {

constexpr int NDT = 256;    // threads per workgroup, one voxel each
constexpr int ND_CAP = 256; // candidates staged in LDS per evaluation round
// Per-axis squared differences of staged candidates over the tile's
// coordinates (orthogonal periods or none): TABN doubles, a chunk of
// TABN / W candidates at a time for W = the sum of the tile's sides.
constexpr int TABN = 2048;
constexpr int TABW = 64;    // largest W that uses the table
// Orthogonal search: the sorted positions of one batch of bins' sites, one
// per slot, SLOTCAP at a time (one site per thread and pass).
constexpr int SLOTCAP = 1024;
constexpr int kNdGrid = 8192;

__device__ inline unsigned long long nd_ordered(double v)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ inline double nd_from_ordered(unsigned long long u)
{
    unsigned long long b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)b);
}

__device__ inline unsigned long long wave_max_u64(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}

// Fractional coordinate i of Cartesian point s (general periods).
__device__ inline double frac_coord(const NdDev& J, int nd, const double* s, int i)
{
    double f = 0.0;
    for (int a = 0; a < nd; ++a)
        f += J.Pinv[i][a] * s[a];
    return f;
}

// ------------------------------------------------------------------ binning

// One thread per site.  Invalid sites are ORed into status_acc (a zeroed
// word; k_nd_scatter publishes it).  The kernel also sets clear_words words
// at `clear` to zero (the next call's zeroed scratch), if given.
__global__ __launch_bounds__(NDT) void k_nd_count(NdDev J, int32_t* status_acc, int32_t* clear, int64_t clear_words)
{
    const int64_t i = blockIdx.x * (int64_t)NDT + threadIdx.x;
    if (clear) {
        const int64_t stride = (int64_t)gridDim.x * NDT, nq = clear_words / 4;
        int4* q = (int4*)clear;
        for (int64_t k = i; k < nq; k += stride)
            q[k] = make_int4(0, 0, 0, 0);
    }
    const bool live = i < J.nsites;
    unsigned long long hi = 0ull, lo = 0ull, mag = 0ull;
    if (live) {
        const int nd = J.ndim;
        bool ok = true;
        int64_t lin = 0, stride = 1;
        double s[kMaxDim];
        for (int a = 0; a < nd; ++a) {
            s[a] = J.coords[i * nd + a];
            // sites taken as they are (period vectors): within the scale
            // bound, so that the rounding margin stays finite
            ok = ok && (J.lattice ? fabs(s[a]) <= VT_SCALE_MAX : isfinite(s[a]));
        }
        for (int a = 0; a < nd; ++a) {
            int b = 0;
            if (J.lattice) {
                if (ok) {
                    const double f = frac_coord(J, nd, s, a);
                    const double r = f - floor(f);
                    const int v = (int)(r * J.inv_bs[a]);
                    b = v < 0 ? 0 : (v >= J.nb[a] ? J.nb[a] - 1 : v);
                    const unsigned long long m = nd_ordered(fabs(s[a]));
                    mag = m > mag ? m : mag;
                }
            } else {
                double c = s[a];
                if (J.bc && isfinite(c))
                    c = cell_coord(c, J.L[a]);
                if (!(c >= 0.0 && c < J.L[a])) {
                    ok = false;
                } else {
                    const int v = (int)(c * J.inv_bs[a]);
                    b = v < 0 ? 0 : (v >= J.nb[a] ? J.nb[a] - 1 : v);
                }
            }
            lin += b * stride;
            stride *= J.nb[a];
        }
        if (J.kind != KIND_VORONOI) {
            const double p = J.param[i];
            if (!(fabs(p) <= VT_SCALE_MAX)) {  // also true for NaN
                ok = false;
            } else {
                hi = nd_ordered(p);
                lo = nd_ordered(-p);
            }
        }
        if (!ok) {
            lin = 0;
            hi = lo = mag = 0ull;
            atomicOr(status_acc, ST_INPUT);
        }
        J.site_bin[i] = (int32_t)lin;
        J.site_rank[i] = atomicAdd(&J.bin_count[lin], 1);
    }
    // parameter and coordinate bounds: one atomic per wavefront
    hi = wave_max_u64(hi);
    lo = wave_max_u64(lo);
    mag = wave_max_u64(mag);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        if (hi)
            atomicMax(&J.pbound[0], hi);
        if (lo)
            atomicMax(&J.pbound[1], lo);
        if (mag)
            atomicMax(&J.pbound[2], mag);
    }
}

// Thread 0 also publishes the status that k_nd_count accumulated.
__global__ __launch_bounds__(NDT) void k_nd_scatter(NdDev J, const int32_t* __restrict__ status_acc)
{
    const int64_t i = blockIdx.x * (int64_t)NDT + threadIdx.x;
    if (i >= J.nsites)
        return;
    if (i == 0)
        *J.status = *status_acc;
    const int nd = J.ndim;
    const int64_t pos = J.bin_start[J.site_bin[i]] + J.site_rank[i];
    double s[kMaxDim];
    for (int a = 0; a < nd; ++a)
        s[a] = J.coords[i * nd + a];
    for (int a = 0; a < nd; ++a) {
        if (J.lattice) {
            J.sc[pos * nd + a] = s[a];
            J.sf[pos * nd + a] = frac_coord(J, nd, s, a);
        } else {
            J.sc[pos * nd + a] = J.bc ? cell_coord(s[a], J.L[a]) : s[a];
        }
    }
    J.sp[pos] = J.kind != KIND_VORONOI ? J.param[i] : 0.0;
    J.sidx[pos] = (int32_t)i;
}

// ---------------------------------------------------------------- labelling

struct NdConst {
    double M;          // pruning margin
    double pmax, pmin; // parameter range
    double rv;         // 1 / v
};

// What the bounds need of a tile.
template <int D>
struct NdTile {
    double lo[D], hi[D];     // orthogonal: box of voxel centres; lattice: fractional box
    double blo[D], bhi[D];   // lattice: Cartesian bounding box of the voxel centres
    double cen[D];           // lattice: fractional centre
};

// Staged candidates.  For general periods each carries the box of
// translations k (first value and count per axis) to evaluate.
template <int D, bool LAT>
struct NdLds {
    double c[D][ND_CAP];
    double klo[LAT ? D : 1][LAT ? ND_CAP : 1];
    double off[LAT ? D : 1][LAT ? ND_CAP : 1];  // single-translation candidates: k_0 L_0a + k_1 L_1a + ...
    int32_t sgl[LAT ? ND_CAP : 1];              // the candidate's box holds one translation
    int32_t kn[LAT ? D : 1][LAT ? ND_CAP : 1];
    double p[ND_CAP];
    int32_t idx[ND_CAP];
    int32_t dead[ND_CAP];    // beaten on the whole tile by the reference site
    double tab[LAT || D < 2 ? 1 : TABN];  // [candidate of the chunk][row]: d_a * d_a
    double kl[ND_CAP];                    // lower bound of each staged candidate's key over the tile
    int32_t slot[SLOTCAP];                // sorted site positions of the current batch
    int32_t count;
    int32_t sovf;                         // the search staged more than ND_CAP candidates
    double geo[LAT ? D * (D + 2) + 1 : 1]; // general periods: reference image, tile centre, half edges, parameter
    NdTile<D> tile;                       // general periods: the current tile's geometry
    double red[NDT / WAVE];
    int32_t ired[NDT / WAVE];
};

// Smallest v over the workgroup and a `pos` that attains it.
template <class L>
__device__ inline double block_argmin(double v, int pos, L& S, int& at)
{
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o);
        const int q = __shfl_xor(pos, o);
        if (w < v || (w == v && q < pos)) {
            v = w;
            pos = q;
        }
    }
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        S.red[threadIdx.x / WAVE] = v;
        S.ired[threadIdx.x / WAVE] = pos;
    }
    __syncthreads();
    double r = S.red[0];
    at = S.ired[0];
    for (int w = 1; w < NDT / WAVE; ++w)
        if (S.red[w] < r) {
            r = S.red[w];
            at = S.ired[w];
        }
    return r;
}

// Exclusive prefix sum of v over the workgroup; total = the sum.
template <class L>
__device__ inline int block_excl_scan(int v, int& total, L& S)
{
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    int x = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    __syncthreads();
    if (lane == WAVE - 1)
        S.ired[w] = x;
    __syncthreads();
    int off = 0;
    total = 0;
    for (int k = 0; k < NDT / WAVE; ++k) {
        const int t = S.ired[k];
        off += k < w ? t : 0;
        total += t;
    }
    return off + x - v;
}

template <class L>
__device__ inline int block_max_int(int v, L& S)
{
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0)
        S.ired[threadIdx.x / WAVE] = v;
    __syncthreads();
    int r = S.ired[0];
    for (int w = 1; w < NDT / WAVE; ++w)
        r = max(r, S.ired[w]);
    return r;
}

// The next mixed-radix digit of rem in base d (rem becomes rem / d), in
// 32-bit arithmetic whenever both fit (always, for tile indices below 2^32).
__device__ inline int64_t take_digit(int64_t& rem, int64_t d)
{
    if (rem < 0x100000000LL && d < 0x100000000LL) {
        const unsigned r = (unsigned)rem, dd = (unsigned)d;
        const unsigned q = r / dd;
        rem = q;
        return (int64_t)(r - q * dd);
    }
    const int64_t q = rem / d, o = rem - q * d;
    rem = q;
    return o;
}

// Key of a squared distance q (bounds only: Johnson-Mehl through 1/v).
template <int KIND>
__device__ inline double key_of_q(double q, double p, const NdConst& C)
{
    if (KIND == KIND_VORONOI)
        return q;
    if (KIND == KIND_LAGUERRE)
        return q - p;
    return p + sqrt(q) * C.rv;
}


// Bounds of the key of the sorted site `pos` over the tile (orthogonal
// periods or none): per axis the smallest and largest (minimum-image)
// distance to the box of voxel centres, then the key of the kind.
template <int KIND, int DIM>
__device__ inline void site_bounds(const NdDev& J, const NdConst& C, int64_t pos, const NdTile<DIM>& G,
                                   double& kl, double& ku)
{
    double lq = 0.0, uq = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double s = J.sc[pos * DIM + a];
        double dmin, dmax;
        if (!J.bc) {
            dmin = fmax(0.0, fmax(G.lo[a] - s, s - G.hi[a]));
            dmax = fmax(fabs(s - G.lo[a]), fabs(s - G.hi[a]));
        } else {
            // the image nearest the centre c of [lo, hi]: no other image comes
            // nearer to the interval (c is at most L/2 from it, every other
            // image at least L/2), and from it no voxel of the interval is
            // farther than |s - c| + half width (nor than L/2, the largest
            // minimum-image distance)
            const double c = 0.5 * (G.lo[a] + G.hi[a]), hw = 0.5 * (G.hi[a] - G.lo[a]);
            double e = fabs(s - c);
            e = fmin(e, J.L[a] - e);
            dmin = fmax(0.0, e - hw);
            dmax = fmin(e + hw, J.H[a]);
        }
        lq += dmin * dmin;
        uq += dmax * dmax;
    }
    const double p = J.sp[pos];
    kl = key_of_q<KIND>(lq, p, C);
    ku = key_of_q<KIND>(uq, p, C);
}

// Cartesian image of sorted site `pos` under translation k (approximate:
// bounds only).
template <int DIM>
__device__ inline void lattice_image(const NdDev& J, int64_t pos, const double* k, double* img)
{
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double o = 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i)
            o += k[i] * J.P[i][a];
        img[a] = J.sc[pos * DIM + a] + o;
    }
}

// Squared distance bounds between a point and the tile's Cartesian box.
template <int DIM>
__device__ inline void box_q(const NdTile<DIM>& G, const double* y, double& lq, double& uq)
{
    lq = 0.0;
    uq = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double dmin = fmax(0.0, fmax(G.blo[a] - y[a], y[a] - G.bhi[a]));
        const double dmax = fmax(fabs(y[a] - G.blo[a]), fabs(y[a] - G.bhi[a]));
        lq += dmin * dmin;
        uq += dmax * dmax;
    }
}

// General periods: upper bound of the key of sorted site `pos` over the tile,
// through the translation that brings it nearest the tile's centre.
template <int KIND, int DIM>
__device__ inline double lattice_upper(const NdDev& J, const NdConst& C, int64_t pos, const NdTile<DIM>& G)
{
    double k[DIM], img[DIM], lq, uq;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
        k[i] = rint(G.cen[i] - J.sf[pos * DIM + i]);
    lattice_image<DIM>(J, pos, k, img);
    box_q<DIM>(G, img, lq, uq);
    return key_of_q<KIND>(uq, J.sp[pos], C);
}

// The visited bin box: the tile's bins [bl, bh] grown by elo bins below and
// ehi bins above along each axis.  Per axis the first bin (unwrapped) and the
// width; full = the axis is covered entirely.
struct NdBox {
    int first[kMaxDim], width[kMaxDim];
    bool full[kMaxDim];
    int64_t count;
};

template <int DIM>
__device__ inline NdBox grown_box(const NdDev& J, const int* bl, const int* bh, const int* elo, const int* ehi)
{
    NdBox B;
    B.count = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int f = bl[a] - elo[a], e = bh[a] + ehi[a];
        if (J.bc) {
            B.full[a] = e - f + 1 >= J.nb[a];
            if (B.full[a]) {
                f = 0;
                e = J.nb[a] - 1;
            }
        } else {
            f = max(f, 0);
            e = min(e, J.nb[a] - 1);
            B.full[a] = f == 0 && e == J.nb[a] - 1;
        }
        B.first[a] = f;
        B.width[a] = e - f + 1;
        B.count *= B.width[a];
    }
    return B;
}

// Bin j (0 <= j < B.count) of box B: its linear bin index, and whether it
// lies inside box P as well (P the previous ring; has_prev false for ring 0).
template <int DIM>
__device__ inline int64_t box_bin(const NdDev& J, const NdBox& B, int64_t j, const NdBox& P, bool has_prev,
                                  bool& inside_prev)
{
    int64_t lin = 0, stride = 1;
    bool in = has_prev;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int w = B.width[a];
        const int o = (int)(j % w);
        j /= w;
        int b = B.first[a] + o;
        const int nb = J.nb[a];
        b = ((b % nb) + nb) % nb;
        if (in && !P.full[a]) {
            const int rel = (((b - P.first[a]) % nb) + nb) % nb;
            in = rel < P.width[a];
        }
        lin += b * stride;
        stride *= nb;
    }
    inside_prev = in;
    return lin;
}

// box_bin in 32-bit arithmetic, for the orthogonal search.  A box that does
// not cover an axis is narrower than the bin grid and starts above -nb, so
// its bins lie in (-nb, 2 nb) before wrapping; a box that covers an axis
// starts at 0.  (The bin count fits in 32 bits.)
template <int DIM>
__device__ inline int box_bin32(const NdDev& J, const NdBox& B, int j, const NdBox& P, bool has_prev,
                                bool& inside_prev)
{
    int lin = 0, stride = 1;
    bool in = has_prev;
    unsigned u = (unsigned)j;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned w = (unsigned)B.width[a];
        const unsigned q = u / w;
        const int o = (int)(u - q * w);
        u = q;
        const int nb = J.nb[a];
        int b = B.first[a] + o;
        b = b < 0 ? b + nb : (b >= nb ? b - nb : b);
        if (in && !P.full[a]) {
            int rel = b - P.first[a];
            rel = rel < 0 ? rel + nb : (rel >= nb ? rel - nb : rel);
            in = rel < P.width[a];
        }
        lin += b * stride;
        stride *= nb;
    }
    inside_prev = in;
    return lin;
}

// General periods grow whole rings: the box of ring r, and the smallest
// Cartesian distance from the tile to a site outside it (infinite once every
// site has been visited): a fractional gap gamma along axis a is at least
// gamma / |row a of Pinv| in Cartesian distance.
template <int DIM>
__device__ inline NdBox ring_box(const NdDev& J, const int* bl, const int* bh, int r)
{
    int e[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        e[a] = r;
    return grown_box<DIM>(J, bl, bh, e, e);
}

template <int DIM>
__device__ inline double ring_gap(const NdDev& J, const NdBox& B, const NdTile<DIM>& G)
{
    double g = __builtin_inf();
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (B.full[a])
            continue;
        const double low = G.lo[a] - (double)B.first[a] * J.bs[a];
        const double high = (double)(B.first[a] + B.width[a]) * J.bs[a] - G.hi[a];
        g = fmin(g, fmax(fmin(low, high), 0.0) / J.rown[a]);
    }
    return g;
}

// Orthogonal periods or none: distances from the tile to the sites beyond
// the low and high faces of the visited box along axis a (infinite where no
// site lies beyond).  On a periodic axis that is not covered entirely, the
// sites beyond either face are the same ones, seen through the two nearest
// periods, so each face gap only bounds them together with the other.
template <int DIM>
__device__ inline void face_gaps(const NdDev& J, const NdBox& B, const NdTile<DIM>& G, int a, double& glo,
                                 double& ghi)
{
    glo = ghi = __builtin_inf();
    const double low = G.lo[a] - (double)B.first[a] * J.bs[a];
    const double high = (double)(B.first[a] + B.width[a]) * J.bs[a] - G.hi[a];
    if (J.bc) {
        if (B.full[a])
            return;
        glo = fmax(low, 0.0);
        ghi = fmax(high, 0.0);
    } else {
        if (B.first[a] > 0)
            glo = fmax(low, 0.0);
        if (B.first[a] + B.width[a] < J.nb[a])
            ghi = fmax(high, 0.0);
    }
}

// Voronoi and Laguerre, orthogonal periods or none: true when the reference
// site (ce = its coordinates, pr its parameter) beats staged candidate k by
// more than M at every voxel centre of the tile.  With images that stay the
// same over the tile, the difference of the two keys is, along each axis,
// (x - e)^2 - (x - r)^2, linear in x, so its minimum over [lo, hi] is at an
// end; the sum of those minima bounds the difference from below.
template <int KIND, int DIM, bool LAT>
__device__ inline bool beaten_on_tile(const NdDev& J, const NdConst& C, const NdTile<DIM>& G,
                                      const NdLds<DIM, LAT>& S, int k, const double* cr, double pr)
{
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double e = S.c[a][k], r = cr[a];
        if (J.bc) {
            // nearest images to the tile's centre, kept only when each is the
            // minimum image for every voxel of the tile
            const double c = 0.5 * (G.lo[a] + G.hi[a]), hw = 0.5 * (G.hi[a] - G.lo[a]);
            const double lim = J.H[a] * (1.0 - 0x1p-30);
            double de = e - c, dr = r - c;
            de = de >= J.H[a] ? de - J.L[a] : (de < -J.H[a] ? de + J.L[a] : de);
            dr = dr >= J.H[a] ? dr - J.L[a] : (dr < -J.H[a] ? dr + J.L[a] : dr);
            if (!(fabs(de) + hw < lim && fabs(dr) + hw < lim))
                return false;
            e = c + de;
            r = c + dr;
        }
        const double vlo = (G.lo[a] - e) * (G.lo[a] - e) - (G.lo[a] - r) * (G.lo[a] - r);
        const double vhi = (G.hi[a] - e) * (G.hi[a] - e) - (G.hi[a] - r) * (G.hi[a] - r);
        acc += fmin(vlo, vhi);
    }
    if (KIND == KIND_LAGUERRE)
        acc -= S.p[k] - pr;
    return acc > C.M;
}

// Marks the staged candidates [0, cnt) that cannot win.  Orthogonal periods
// or none: with use_cut, those whose lower bound exceeds cut (staged while
// the search's UB was larger); for Voronoi and Laguerre, those that the
// reference site beats on the whole tile.  General periods (Voronoi and
// Laguerre): candidates with a single translation that the reference's image
// nearest the tile beats on the whole parallelepiped of voxel centres (centre
// c, half edges u_i); for images e and r, |x - e|^2 - |x - r|^2 =
// (r - e) . (2x - e - r) is linear in x, so its minimum there is
// (r - e) . (2c - e - r) - 2 sum_i |(r - e) . u_i|.  The reference is staged
// with that translation (its lower bound is below UB), so the winner's
// computed key is at most that image's.
template <int KIND, int DIM, bool LAT>
__device__ inline void mark_beaten(const NdDev& J, const NdConst& C, const NdTile<DIM>& G, NdLds<DIM, LAT>& S,
                                   int cnt, int ref, bool use_cut, double cut, const int64_t* v0, const int64_t* ve)
{
    if (LAT) {
        // the reference's image r, the centre c and the half edges u_i of the
        // tile go to LDS (geo: r, c, u_0, u_1, ..., parameter of r)
        const bool use = KIND != KIND_JM && ref >= 0;
        double* g = S.geo;
        __syncthreads();
        if (use && threadIdx.x == 0) {
            double kr[DIM], r[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i)
                kr[i] = rint(G.cen[i] - J.sf[(int64_t)ref * DIM + i]);
            lattice_image<DIM>(J, ref, kr, r);
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                g[a] = r[a];
                g[DIM + a] = 0.0;
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                const double mid = 0.5 * ((double)v0[i] + (double)ve[i]) + 0.5;
                const double half = 0.5 * (double)(ve[i] - v0[i]);
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    g[DIM + a] += mid * J.hv[i][a];
                    g[(2 + i) * DIM + a] = half * J.hv[i][a];
                }
            }
            g[DIM * (DIM + 2)] = J.sp[ref];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < cnt; k += NDT) {
            bool d = use_cut && S.kl[k] > cut;
            bool single = use && !d;
#pragma unroll
            for (int i = 0; i < DIM; ++i)
                single = single && S.kn[LAT ? i : 0][LAT ? k : 0] == 1;
            if (single) {
                double dl[DIM], lin = 0.0, slope = 0.0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    double o = 0.0;
#pragma unroll
                    for (int i = 0; i < DIM; ++i)
                        o += S.klo[LAT ? i : 0][LAT ? k : 0] * J.P[i][a];
                    const double e = S.c[a][k] + o;
                    dl[a] = g[a] - e;
                    lin += dl[a] * (2.0 * g[DIM + a] - e - g[a]);
                }
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    double t = 0.0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a)
                        t += dl[a] * g[(2 + i) * DIM + a];
                    slope += fabs(t);
                }
                double acc = lin - 2.0 * slope;
                if (KIND == KIND_LAGUERRE)
                    acc -= S.p[k] - g[DIM * (DIM + 2)];
                d = acc > C.M;
            }
            S.dead[k] = d;
        }
        __syncthreads();
        return;
    }
    double cr[DIM];
    double pr = 0.0;
    const bool use = KIND != KIND_JM && ref >= 0;
    if (use) {
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            cr[a] = J.sc[(int64_t)ref * DIM + a];
        pr = J.sp[ref];
    }
    for (int k = threadIdx.x; k < cnt; k += NDT) {
        bool d = use_cut && S.kl[k] > cut;
        if (!d && use)
            d = beaten_on_tile<KIND, DIM, LAT>(J, C, G, S, k, cr, pr);
        S.dead[k] = d;
    }
    __syncthreads();
}

// The exact key of staged candidate k at voxel centre x (the operations of
// the definition in the file comment).
template <int KIND>
__device__ inline double nd_key_q(const NdDev& J, double q, double p)
{
    if (KIND == KIND_VORONOI)
        return q;
    if (KIND == KIND_LAGUERRE)
        return q - p;
    return J.jm_div ? p + key_sqrt(q) / J.growth : p + key_sqrt(q) * J.rgrowth;
}

// General periods: for a staged candidate whose box holds one translation k,
// the offset k_0 L_0a + k_1 L_1a + ... of every axis, formed as nd_key forms
// it (same operations, same order), so that the evaluation adds it instead
// of forming it at every voxel.
template <int DIM, bool LAT>
__device__ inline void lattice_offsets(const NdDev& J, NdLds<DIM, LAT>& S, int slot, const double* klo, const int* kn)
{
    if (!LAT)
        return;
    bool one = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        one = one && kn[a] == 1;
    S.sgl[LAT ? slot : 0] = one;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double o = klo[0] * J.P[0][a];
#pragma unroll
        for (int i = 1; i < DIM; ++i)
            o = o + klo[i] * J.P[i][a];
        S.off[LAT ? a : 0][LAT ? slot : 0] = o;
    }
}

template <int KIND, int DIM, bool LAT>
__device__ inline double nd_key(const NdDev& J, const NdLds<DIM, LAT>& S, int k, const double* x)
{
    double q;
    if (!LAT) {
        double d[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double e = S.c[a][k] - x[a];
            if (J.bc)
                e = e >= J.H[a] ? e - J.L[a] : (e < -J.H[a] ? e + J.L[a] : e);
            d[a] = e;
        }
        q = d[0] * d[0];
        if (DIM > 1) {
            double T = d[1] * d[1];
#pragma unroll
            for (int a = 2; a < DIM; ++a)
                T = T + d[a] * d[a];
            q = q + T;
        }
    } else {
        double e[DIM], kk[DIM];
        int cnt[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            e[a] = S.c[a][k] - x[a];
            kk[a] = S.klo[LAT ? a : 0][LAT ? k : 0];
            cnt[a] = 0;
        }
        q = __builtin_inf();
        for (;;) {
            double d[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                double o = kk[0] * J.P[0][a];
#pragma unroll
                for (int i = 1; i < DIM; ++i)
                    o = o + kk[i] * J.P[i][a];
                d[a] = e[a] + o;
            }
            double qk = d[0] * d[0];
            if (DIM > 1) {
                double T = d[1] * d[1];
#pragma unroll
                for (int a = 2; a < DIM; ++a)
                    T = T + d[a] * d[a];
                qk = qk + T;
            }
            q = fmin(q, qk);
            // next translation of the box (the same for every thread)
            int i = 0;
            for (; i < DIM; ++i) {
                if (++cnt[i] < S.kn[LAT ? i : 0][LAT ? k : 0]) {
                    kk[i] += 1.0;
                    break;
                }
                cnt[i] = 0;
                kk[i] = S.klo[LAT ? i : 0][LAT ? k : 0];
            }
            if (i == DIM)
                break;
        }
    }
    return nd_key_q<KIND>(J, q, S.p[k]);
}

// Evaluates the staged candidates [0, count) at the thread's VPT voxels
// (orthogonal periods: voxel j is x moved by j * tx0 voxels along axis 0,
// with axis-0 coordinate x0s[j]; general periods: one voxel, x).  With
// orthogonal periods the terms of axes 1 .. DIM-1 are the same for every
// voxel of the thread and are summed once, in the order of the definition.
template <int KIND, int DIM, bool LAT, int VPT>
__device__ inline void nd_evaluate(const NdDev& J, const NdLds<DIM, LAT>& S, int count, const double* x,
                                   const double* x0s, double* best, int* blab)
{
    for (int k = 0; k < count; ++k) {
        if (S.dead[k])  // the same for every thread
            continue;
        const int id = S.idx[k];
        double key[VPT];
        if (LAT) {
            if (S.sgl[LAT ? k : 0]) {
                // one translation: d_a = (s_a - x_a) + offset_a, folded as in nd_key
                double d[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a)
                    d[a] = (S.c[a][k] - x[a]) + S.off[LAT ? a : 0][LAT ? k : 0];
                double q = d[0] * d[0];
                if (DIM > 1) {
                    double T = d[1] * d[1];
#pragma unroll
                    for (int a = 2; a < DIM; ++a)
                        T = T + d[a] * d[a];
                    q = q + T;
                }
                key[0] = nd_key_q<KIND>(J, q, S.p[k]);
            } else {
                key[0] = nd_key<KIND, DIM, LAT>(J, S, k, x);
            }
        } else {
            double T = 0.0;
#pragma unroll
            for (int a = 1; a < DIM; ++a) {
                double e = S.c[a][k] - x[a];
                if (J.bc)
                    e = e >= J.H[a] ? e - J.L[a] : (e < -J.H[a] ? e + J.L[a] : e);
                T = a == 1 ? e * e : T + e * e;
            }
            const double p = S.p[k];
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                double e = S.c[0][k] - x0s[j];
                if (J.bc)
                    e = e >= J.H[0] ? e - J.L[0] : (e < -J.H[0] ? e + J.L[0] : e);
                key[j] = nd_key_q<KIND>(J, DIM > 1 ? e * e + T : e * e, p);
            }
        }
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
            if (key[j] < best[j] || (key[j] == best[j] && id < blab[j])) {
                best[j] = key[j];
                blab[j] = id;
            }
        }
    }
}

// Where a thread builds and reads the per-axis table (orthogonal periods or
// none, 2 to 6 axes): row r = offset of axis a + tile-local coordinate i holds
// d_a * d_a for the voxel coordinate x_a = (v0_a + i + 1/2) h_a, d_a the
// (minimum-image) difference s_a - x_a of each candidate of the chunk.  The
// key then sums the rows of the thread's voxel in the definition's order,
// q = d0*d0 + T with T = d1*d1, T + d2*d2, ...: the same operations as
// nd_evaluate, each difference and square computed once per tile instead of
// once per voxel.
struct NdTab {
    bool on;        // the table is used for this tile
    int W;          // rows: the sum of the tile's sides
    int row[kMaxDim];  // the thread's rows (its first voxel)
    int brow;       // the row this thread builds, and its axis
    int baxis;
    int bk0, bkstep;   // first candidate of the chunk it builds, stride
    double bx;      // the voxel coordinate of its row
};

template <int KIND, int DIM, bool LAT, int VPT>
__device__ inline void nd_eval_round(const NdDev& J, NdLds<DIM, LAT>& S, int cnt, const NdTab& tb, int tx0,
                                     const double* x, const double* x0s, bool live_any, double* best, int* blab)
{
    if (LAT || DIM < 2 || !tb.on) {
        if (live_any && cnt > 0)
            nd_evaluate<KIND, DIM, LAT, VPT>(J, S, cnt, x, x0s, best, blab);
        return;
    }
    const int W = tb.W;
    const int chunk = TABN / W;
    for (int c0 = 0; c0 < cnt; c0 += chunk) {
        const int nk = min(chunk, cnt - c0);
        if (tb.bk0 >= 0) {
            const double Ha = J.H[tb.baxis], La = J.L[tb.baxis];
            for (int k = tb.bk0; k < nk; k += tb.bkstep) {
                double e = S.c[tb.baxis][c0 + k] - tb.bx;
                if (J.bc)
                    e = e >= Ha ? e - La : (e < -Ha ? e + La : e);
                S.tab[LAT || DIM < 2 ? 0 : k * W + tb.brow] = e * e;
            }
        }
        __syncthreads();
        if (live_any) {
            for (int k = 0; k < nk; ++k) {
                const int g = c0 + k;
                if (S.dead[g])  // the same for every thread
                    continue;
                const double* t = &S.tab[LAT || DIM < 2 ? 0 : k * W];
                double T = t[tb.row[1]];
#pragma unroll
                for (int a = 2; a < DIM; ++a)
                    T = T + t[tb.row[a]];
                const double p = S.p[g];
                const int id = S.idx[g];
#pragma unroll
                for (int j = 0; j < VPT; ++j) {
                    const double key = nd_key_q<KIND>(J, t[tb.row[0] + j * tx0] + T, p);
                    if (key < best[j] || (key == best[j] && id < blab[j])) {
                        best[j] = key;
                        blab[j] = id;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// General periods: the box of translations k that can bring sorted site
// `pos` within key `cut` of the tile.  Returns false when none can.
template <int KIND, int DIM>
__device__ inline bool lattice_reach(const NdDev& J, const NdConst& C, int64_t pos, const NdTile<DIM>& G,
                                     double cut, double* klo, int* kn, double& klow)
{
    klow = -__builtin_inf();  // unknown unless the box is trimmed below
    const double p = J.sp[pos];
    double qmax;  // largest squared distance at which the key stays <= cut
    if (KIND == KIND_VORONOI)
        qmax = cut;
    else if (KIND == KIND_LAGUERRE)
        qmax = cut + p;
    else
        qmax = cut >= p ? ((cut - p) * J.growth) * ((cut - p) * J.growth) : -1.0;
    if (!(qmax >= 0.0))
        return false;
    const double R = sqrt(qmax) * (1.0 + 0x1p-20);
    double lo[DIM];
    int64_t total = 1;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        const double f = J.sf[pos * DIM + i];
        const double rho = R * J.rown[i] * (1.0 + 0x1p-20) + 0x1p-30 * (1.0 + fabs(f));
        const double a = ceil(G.lo[i] - rho - f), b = floor(G.hi[i] + rho - f);
        if (a > b)
            return false;
        lo[i] = a;
        kn[i] = (int)fmin(b - a + 1.0, 1048576.0);
        total = total * kn[i] < ((int64_t)1 << 40) ? total * kn[i] : ((int64_t)1 << 40);
    }
    // keep only the translations whose image can come within reach of the
    // tile's box; when the box is large, keep it whole
    if (total <= 4096) {
        double nlo[DIM], nhi[DIM], k[DIM];
        int cnt[DIM];
        bool any = false;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            cnt[i] = 0;
            k[i] = lo[i];
            nlo[i] = __builtin_inf();
            nhi[i] = -__builtin_inf();
        }
        for (;;) {
            double img[DIM], lq, uq;
            lattice_image<DIM>(J, pos, k, img);
            box_q<DIM>(G, img, lq, uq);
            const double kq = key_of_q<KIND>(lq, p, C);
            if (kq <= cut + C.M) {
                any = true;
                klow = klow == -__builtin_inf() ? kq : fmin(klow, kq);
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    nlo[i] = fmin(nlo[i], k[i]);
                    nhi[i] = fmax(nhi[i], k[i]);
                }
            }
            int i = 0;
            for (; i < DIM; ++i) {
                if (++cnt[i] < kn[i]) {
                    k[i] += 1.0;
                    break;
                }
                cnt[i] = 0;
                k[i] = lo[i];
            }
            if (i == DIM)
                break;
        }
        if (!any)
            return false;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            lo[i] = nlo[i];
            kn[i] = (int)(nhi[i] - nlo[i] + 1.0);
        }
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
        klo[i] = lo[i];
    return true;
}

// One round of the search for general periods (the orthogonal search
// inlines the same steps): the bins of box B that are not in P (when
// `grown`) go in batches of NDT; their sites' sorted positions are listed in
// LDS, one thread per site takes the site's upper bound over the tile, UB and
// a site attaining it are reduced, and the sites that can come within
// UB + M are staged right away with their lower bound (and, for general
// periods, their box of translations).  UB only decreases, so the final cut
// is applied to the staged sites afterwards.  More than ND_CAP staged sets
// S.sovf.
template <int KIND, int DIM, bool LAT>
__device__ inline void search_round(const NdDev& J, const NdConst& C, const NdTile<DIM>& G, NdLds<DIM, LAT>& S,
                                    const NdBox& B, const NdBox& P, bool grown, double& UB, int& ubpos)
{
    const int tid = threadIdx.x;
    const int nbox = (int)B.count;
    for (int jb = 0; jb < nbox; jb += NDT) {
        const int j = jb + tid;
        int s0 = 0, n = 0;
        if (j < nbox) {
            bool in_prev;
            const int lin = box_bin32<DIM>(J, B, j, P, grown, in_prev);
            if (!in_prev) {
                s0 = J.bin_start[lin];
                n = J.bin_start[lin + 1] - s0;
            }
        }
        int total;
        const int pre = block_excl_scan(n, total, S);
        for (int w0 = 0; w0 < total; w0 += SLOTCAP) {
            const int k0 = max(0, w0 - pre), k1 = min(n, w0 + SLOTCAP - pre);
            for (int k = k0; k < k1; ++k)
                S.slot[pre + k - w0] = s0 + k;
            __syncthreads();
            const int wn = min(SLOTCAP, total - w0);
            double kls[SLOTCAP / NDT];
            int ps[SLOTCAP / NDT];
            double my = __builtin_inf();
            int mypos = -1;
#pragma unroll
            for (int r = 0; r < SLOTCAP / NDT; ++r) {
                const int i = tid + r * NDT;
                kls[r] = __builtin_inf();
                ps[r] = -1;
                if (i < wn) {
                    const int pos = S.slot[i];
                    double ku;
                    if (LAT) {
                        ku = lattice_upper<KIND, DIM>(J, C, pos, G);
                    } else {
                        double kl;
                        site_bounds<KIND, DIM>(J, C, pos, G, kl, ku);
                        kls[r] = kl;
                    }
                    ps[r] = pos;
                    if (ku < my) {
                        my = ku;
                        mypos = pos;
                    }
                }
            }
            int at;
            const double m = block_argmin(my, mypos, S, at);
            if (m < UB) {
                UB = m;
                ubpos = at;
            }
            const double cutr = UB + C.M;
#pragma unroll
            for (int r = 0; r < SLOTCAP / NDT; ++r) {
                if (ps[r] < 0)
                    continue;
                const int64_t pos = ps[r];
                double klo[DIM], klw = kls[r];
                int kn[DIM];
                const bool keep = LAT ? lattice_reach<KIND, DIM>(J, C, pos, G, cutr, klo, kn, klw) : klw <= cutr;
                if (keep) {
                    const int slot = atomicAdd(&S.count, 1);
                    if (slot < ND_CAP) {
#pragma unroll
                        for (int a = 0; a < DIM; ++a)
                            S.c[a][slot] = J.sc[pos * DIM + a];
                        if (LAT) {
#pragma unroll
                            for (int a = 0; a < DIM; ++a) {
                                S.klo[LAT ? a : 0][LAT ? slot : 0] = klo[a];
                                S.kn[LAT ? a : 0][LAT ? slot : 0] = kn[a];
                            }
                            lattice_offsets<DIM, LAT>(J, S, slot, klo, kn);
                        }
                        S.p[slot] = J.sp[pos];
                        S.idx[slot] = J.sidx[pos];
                        S.kl[slot] = klw;
                    } else {
                        S.sovf = 1;
                    }
                }
            }
            __syncthreads();  // the slot list is rewritten next
        }
    }
}

// Four waves per SIMD, except Laguerre and Johnson-Mehl with orthogonal
// periods, whose kernels spill more and run faster with three (5D -31 %, 4D
// Laguerre -4 %; general periods were 7 % slower with three).
template <int KIND, int DIM, bool LAT, int VPT>
__global__ __launch_bounds__(NDT, (KIND == KIND_VORONOI || LAT) ? 4 : 3) void k_nd_label(NdDev J)
{
    __shared__ NdLds<DIM, LAT> S;
    const int tid = threadIdx.x;
    const bool bad = *(volatile int32_t*)J.status != 0;
    NdConst C;
    {
        C.rv = J.rgrowth;
        C.pmax = C.pmin = 0.0;
        if (KIND != KIND_VORONOI && !bad) {
            C.pmax = nd_from_ordered(J.pbound[0]);
            C.pmin = -nd_from_ordered(J.pbound[1]);
        }
        double S2;  // squared length scale of the computed differences
        if (LAT) {
            const double mag = bad ? 0.0 : nd_from_ordered(J.pbound[2]);
            const double D = sqrt((double)DIM) * (2.0 * mag + 3.0 * J.cell_d);
            S2 = D * D;
        } else {
            S2 = 0.0;
            for (int a = 0; a < DIM; ++a)
                S2 += J.L[a] * J.L[a];
        }
        const double pabs = fmax(fabs(C.pmax), fabs(C.pmin));
        const double scale = KIND == KIND_VORONOI ? S2
                           : KIND == KIND_LAGUERRE ? S2 + 2.0 * pabs
                                                   : sqrt(S2) * C.rv + 2.0 * pabs;
        C.M = scale * 0x1p-36;
    }
    for (int64_t t = blockIdx.x; t < J.ntiles; t += gridDim.x) {
        int64_t v0[DIM], ve[DIM], vi[DIM];
        double x[DIM];
        int bl[DIM], bh[DIM];
        NdTile<DIM> G0;
        int64_t rem = t;
        int l = tid;
        // threads along axis 0; with VPT voxels per thread (orthogonal
        // periods only) voxel j is j * tx0 voxels further along axis 0
        const int tx0 = J.T[0] / VPT;
        bool live = true, livev[VPT];
#pragma unroll
        for (int j = 0; j < VPT; ++j)
            livev[j] = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t tc = take_digit(rem, J.nt[a]);
            v0[a] = tc * J.T[a];
            ve[a] = (v0[a] + J.T[a] < J.n[a] ? v0[a] + J.T[a] : J.n[a]) - 1;
            const int ta = a == 0 ? tx0 : J.T[a];
            const int off = l % ta;
            l /= ta;
            vi[a] = v0[a] + off;
            live = live && vi[a] <= ve[a];
#pragma unroll
            for (int j = 0; j < VPT; ++j)
                livev[j] = livev[j] && vi[a] + (a == 0 ? j * tx0 : 0) <= ve[a];
            if (LAT) {
                G0.lo[a] = ((double)v0[a] + 0.5) / (double)J.n[a];
                G0.hi[a] = ((double)ve[a] + 0.5) / (double)J.n[a];
                G0.cen[a] = 0.5 * (G0.lo[a] + G0.hi[a]);
            } else {
                G0.lo[a] = ((double)v0[a] + 0.5) * J.h[a];
                G0.hi[a] = ((double)ve[a] + 0.5) * J.h[a];
                x[a] = ((double)vi[a] + 0.5) * J.h[a];
            }
            const int b0 = (int)(G0.lo[a] * J.inv_bs[a]), b1 = (int)(G0.hi[a] * J.inv_bs[a]);
            bl[a] = min(max(b0, 0), J.nb[a] - 1);
            bh[a] = min(max(b1, 0), J.nb[a] - 1);
        }
        double x0s[VPT];  // axis-0 coordinates of the thread's voxels (orthogonal periods)
#pragma unroll
        for (int j = 0; j < VPT; ++j)
            x0s[j] = LAT ? 0.0 : ((double)(vi[0] + j * tx0) + 0.5) * J.h[0];
        if (LAT) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                // the voxel centre, summed as the definition sums it
                double acc = ((double)vi[0] + 0.5) * J.hv[0][a];
#pragma unroll
                for (int i = 1; i < DIM; ++i)
                    acc = acc + ((double)vi[i] + 0.5) * J.hv[i][a];
                x[a] = acc;
                // bounding box of the tile's centres, term by term
                double b0 = 0.0, b1 = 0.0;
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    const double t0 = ((double)v0[i] + 0.5) * J.hv[i][a];
                    const double t1 = ((double)ve[i] + 0.5) * J.hv[i][a];
                    b0 += fmin(t0, t1);
                    b1 += fmax(t0, t1);
                }
                G0.blo[a] = b0;
                G0.bhi[a] = b1;
            }
        }
        live = live && l == 0;
        bool live_any = false;
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
            livev[j] = livev[j] && l == 0;
            live_any = live_any || livev[j];
        }
        // general periods: the tile's geometry lives in LDS (read where the
        // bounds need it) rather than in registers
        if (LAT) {
            if (tid == 0)
                S.tile = G0;
            __syncthreads();
        }
        const NdTile<DIM>& G = LAT ? S.tile : G0;
        NdTab tb;
        tb.on = false;
        tb.W = 0;
        tb.bk0 = -1;
        tb.bkstep = 1;
        tb.brow = tb.baxis = 0;
        tb.bx = 0.0;
        if (!LAT && DIM >= 2) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                tb.row[a] = tb.W + (int)(vi[a] - v0[a]);
                tb.W += J.T[a];
            }
            tb.on = tb.W <= TABW;
            if (tb.on) {
                // this thread builds row tid % W for candidates tid / W,
                // + 256 / W, ... of each chunk
                const int r = tid % tb.W;
                tb.bkstep = NDT / tb.W;
                tb.bk0 = tid < tb.bkstep * tb.W ? tid / tb.W : -1;
                int i = r, ax = 0;
#pragma unroll
                for (int a = 0; a < DIM - 1; ++a) {
                    if (ax == a && i >= J.T[a]) {
                        i -= J.T[a];
                        ax = a + 1;
                    }
                }
                int64_t va = 0;
                double ha = 0.0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    if (ax == a) {
                        va = v0[a];
                        ha = J.h[a];
                    }
                }
                tb.brow = r;
                tb.baxis = ax;
                tb.bx = ((double)(va + i) + 0.5) * ha;
            }
        }
        double best[VPT];
        int blab[VPT];
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
            best[j] = __builtin_inf();
            blab[j] = 0x7fffffff;
        }
        if (!bad) {
            // 1. grow the box of visited bins until the sites beyond it
            //    provably lose; their keys are at least gap^2, gap^2 - max w
            //    or min t + gap / v for the gap to the box
            double UB = __builtin_inf();
            int ubpos = -1;  // a sorted site attaining UB
            NdBox B, P;
            if (LAT) {
                // general periods: whole rings from the tile's own bins (their
                // staging filter is loose in a skewed cell, so a small box pays)
                int r = 0;
                B = ring_box<DIM>(J, bl, bh, 0);
                P = B;
                if (tid == 0) {
                    S.count = 0;
                    S.sovf = 0;
                }
                for (;;) {
                    search_round<KIND, DIM, LAT>(J, C, G, S, B, P, r > 0, UB, ubpos);
                    const double g = ring_gap<DIM>(J, B, G);
                    if (g == __builtin_inf())
                        break;
                    const double lb_out = KIND == KIND_VORONOI ? g * g
                                        : KIND == KIND_LAGUERRE ? g * g - C.pmax
                                                                : C.pmin + g * C.rv;
                    if (lb_out > UB + C.M)
                        break;
                    ++r;
                    P = B;
                    B = ring_box<DIM>(J, bl, bh, r);
                }
            } else {
                // orthogonal periods or none: start from the first ring of
                // neighbour bins, which makes UB tight, then move only the
                // faces whose sites might still win.  Each round's new bins
                // go in batches of NDT: their sites' sorted positions are
                // listed in LDS, then one thread per site takes its bounds,
                // UB is reduced, and the sites with a lower bound within
                // UB + M are staged right away (UB only decreases, so the
                // final cut is applied to them afterwards).
                int elo[DIM], ehi[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a)
                    elo[a] = ehi[a] = 1;
                B = grown_box<DIM>(J, bl, bh, elo, ehi);
                P = B;
                bool grown = false;
                if (tid == 0) {
                    S.count = 0;
                    S.sovf = 0;
                }
                for (;;) {
                    const int nbox = (int)B.count;
                    for (int jb = 0; jb < nbox; jb += NDT) {
                        const int j = jb + tid;
                        int s0 = 0, n = 0;
                        if (j < nbox) {
                            bool in_prev;
                            const int lin = box_bin32<DIM>(J, B, j, P, grown, in_prev);
                            if (!in_prev) {
                                s0 = J.bin_start[lin];
                                n = J.bin_start[lin + 1] - s0;
                            }
                        }
                        int total;
                        const int pre = block_excl_scan(n, total, S);
                        for (int w0 = 0; w0 < total; w0 += SLOTCAP) {
                            const int k0 = max(0, w0 - pre), k1 = min(n, w0 + SLOTCAP - pre);
                            for (int k = k0; k < k1; ++k)
                                S.slot[pre + k - w0] = s0 + k;
                            __syncthreads();
                            const int wn = min(SLOTCAP, total - w0);
                            double kls[SLOTCAP / NDT];
                            int ps[SLOTCAP / NDT];
                            double my = __builtin_inf();
                            int mypos = -1;
#pragma unroll
                            for (int r = 0; r < SLOTCAP / NDT; ++r) {
                                const int i = tid + r * NDT;
                                kls[r] = __builtin_inf();
                                ps[r] = -1;
                                if (i < wn) {
                                    const int pos = S.slot[i];
                                    double kl, ku;
                                    site_bounds<KIND, DIM>(J, C, pos, G, kl, ku);
                                    kls[r] = kl;
                                    ps[r] = pos;
                                    if (ku < my) {
                                        my = ku;
                                        mypos = pos;
                                    }
                                }
                            }
                            int at;
                            const double m = block_argmin(my, mypos, S, at);
                            if (m < UB) {
                                UB = m;
                                ubpos = at;
                            }
                            const double cutr = UB + C.M;
#pragma unroll
                            for (int r = 0; r < SLOTCAP / NDT; ++r) {
                                if (ps[r] >= 0 && kls[r] <= cutr) {
                                    const int slot = atomicAdd(&S.count, 1);
                                    if (slot < ND_CAP) {
                                        const int64_t pos = ps[r];
#pragma unroll
                                        for (int a = 0; a < DIM; ++a)
                                            S.c[a][slot] = J.sc[pos * DIM + a];
                                        S.p[slot] = J.sp[pos];
                                        S.idx[slot] = J.sidx[pos];
                                        S.kl[slot] = kls[r];
                                    } else {
                                        S.sovf = 1;
                                    }
                                }
                            }
                            __syncthreads();  // the slot list is rewritten next
                        }
                    }
                    bool grow = false;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        double glo, ghi;
                        face_gaps<DIM>(J, B, G, a, glo, ghi);
                        const double llo = KIND == KIND_VORONOI ? glo * glo
                                         : KIND == KIND_LAGUERRE ? glo * glo - C.pmax
                                                                 : C.pmin + glo * C.rv;
                        const double lhi = KIND == KIND_VORONOI ? ghi * ghi
                                         : KIND == KIND_LAGUERRE ? ghi * ghi - C.pmax
                                                                 : C.pmin + ghi * C.rv;
                        // (an infinite gap has no site beyond it: that face stays)
                        const bool mlo = glo != __builtin_inf() && !(llo > UB + C.M);
                        const bool mhi = ghi != __builtin_inf() && !(lhi > UB + C.M);
                        elo[a] += mlo;
                        ehi[a] += mhi;
                        grow = grow || mlo || mhi;
                    }
                    if (!grow)
                        break;
                    P = B;
                    B = grown_box<DIM>(J, bl, bh, elo, ehi);
                    grown = true;
                }
            }
            // 2. stage the candidates (general periods, or an orthogonal search
            //    that staged more than ND_CAP) and take the lexicographic minimum
            const double cut = UB + C.M;
            const bool staged = !S.sovf;  // uniform: read after the search's last barrier
            __syncthreads();
            if (!staged && tid == 0)
                S.count = 0;
            __syncthreads();
            for (int64_t base = 0; base < (staged ? 0 : B.count); base += NDT) {
                const int64_t j = base + tid;
                int s0 = 0, s1 = 0;
                if (j < B.count) {
                    bool unused;
                    const int64_t lin = box_bin<DIM>(J, B, j, B, false, unused);
                    s0 = J.bin_start[lin];
                    s1 = J.bin_start[lin + 1];
                }
                const int rounds = block_max_int(s1 - s0, S);
                for (int k = 0; k < rounds; ++k) {
                    if (s0 + k < s1) {
                        const int s = s0 + k;
                        bool keep;
                        double klo[DIM];
                        int kn[DIM];
                        if (LAT) {
                            double klw;
                            keep = lattice_reach<KIND, DIM>(J, C, s, G, cut, klo, kn, klw);
                        } else {
                            double kl, ku;
                            site_bounds<KIND, DIM>(J, C, s, G, kl, ku);
                            keep = kl <= cut;
                        }
                        if (keep) {
                            const int slot = atomicAdd(&S.count, 1);
#pragma unroll
                            for (int a = 0; a < DIM; ++a)
                                S.c[a][slot] = J.sc[(int64_t)s * DIM + a];
                            if (LAT) {
#pragma unroll
                                for (int a = 0; a < DIM; ++a) {
                                    S.klo[LAT ? a : 0][LAT ? slot : 0] = klo[a];
                                    S.kn[LAT ? a : 0][LAT ? slot : 0] = kn[a];
                                }
                                lattice_offsets<DIM, LAT>(J, S, slot, klo, kn);
                            }
                            S.p[slot] = J.sp[s];
                            S.idx[slot] = J.sidx[s];
                        }
                    }
                    __syncthreads();
                    const int cnt = S.count;
                    __syncthreads();  // every thread has read the count before the next appends
                    if (cnt > ND_CAP - NDT) {
                        mark_beaten<KIND, DIM, LAT>(J, C, G, S, cnt, ubpos, false, cut, v0, ve);
                        nd_eval_round<KIND, DIM, LAT, VPT>(J, S, cnt, tb, tx0, x, x0s, live_any, best, blab);
                        __syncthreads();
                        if (tid == 0)
                            S.count = 0;
                        __syncthreads();
                    }
                }
            }
            const int cnt = S.count;
            mark_beaten<KIND, DIM, LAT>(J, C, G, S, cnt, ubpos, staged, cut, v0, ve);
            nd_eval_round<KIND, DIM, LAT, VPT>(J, S, cnt, tb, tx0, x, x0s, live_any, best, blab);
            __syncthreads();
        }
        if (live_any) {
            int64_t lin = 0, stride = 1;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                lin += vi[a] * stride;
                stride *= J.n[a];
            }
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                if (livev[j]) {
                    J.labels[lin + j * tx0] = bad ? -1 : blab[j];
                    if (J.keys)
                        J.keys[lin + j * tx0] = bad ? __builtin_nan("") : best[j];
                }
            }
        }
    }
}

// Two voxels per thread only with orthogonal periods in 2 to 4 axes (the
// plan never asks for them elsewhere), so only those kernels are built.
template <int KIND, int DIM, bool LAT>
void launch_nd_kind(const NdDev& J, unsigned g, hipStream_t s)
{
    constexpr bool multi = !LAT && DIM >= 2 && DIM <= 4;
    if (multi && J.vpt == 2)
        k_nd_label<KIND, DIM, LAT, multi ? 2 : 1><<<g, NDT, 0, s>>>(J);
    else
        k_nd_label<KIND, DIM, LAT, 1><<<g, NDT, 0, s>>>(J);
}

template <int DIM, bool LAT>
void launch_nd_dim(const NdDev& J, unsigned g, hipStream_t s)
{
    if (J.kind == KIND_VORONOI)
        launch_nd_kind<KIND_VORONOI, DIM, LAT>(J, g, s);
    else if (J.kind == KIND_LAGUERRE)
        launch_nd_kind<KIND_LAGUERRE, DIM, LAT>(J, g, s);
    else
        launch_nd_kind<KIND_JM, DIM, LAT>(J, g, s);
}

template <bool LAT>
hipError_t launch_nd_lat(const NdDev& J, unsigned g, hipStream_t s)
{
    switch (J.ndim) {
    case 1: launch_nd_dim<1, LAT>(J, g, s); break;
    case 2: launch_nd_dim<2, LAT>(J, g, s); break;
    case 3: launch_nd_dim<3, LAT>(J, g, s); break;
    case 4: launch_nd_dim<4, LAT>(J, g, s); break;
    case 5: launch_nd_dim<5, LAT>(J, g, s); break;
    case 6: launch_nd_dim<6, LAT>(J, g, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_nd_bin_count(const NdDev& J, int32_t* status_acc, int32_t* clear, int64_t clear_words,
                               hipStream_t s)
{
    if (!status_acc || (clear_words & 3) != 0 || ((uintptr_t)clear & 15) != 0)
        return hipErrorInvalidValue;
    const int64_t g = (J.nsites + NDT - 1) / NDT;
    k_nd_count<<<(unsigned)g, NDT, 0, s>>>(J, status_acc, clear, clear_words);
    return hipGetLastError();
}

hipError_t launch_nd_bin_scatter(const NdDev& J, const int32_t* status_acc, hipStream_t s)
{
    if (!status_acc)
        return hipErrorInvalidValue;
    const int64_t g = (J.nsites + NDT - 1) / NDT;
    k_nd_scatter<<<(unsigned)g, NDT, 0, s>>>(J, status_acc);
    return hipGetLastError();
}

hipError_t launch_nd_label(const NdDev& J, hipStream_t s)
{
    const bool multi_ok = !J.lattice && J.ndim >= 2 && J.ndim <= 4;
    if (!(J.vpt == 1 || (multi_ok && J.vpt == 2)) || J.T[0] % J.vpt != 0)
        return hipErrorInvalidValue;
    const unsigned g = (unsigned)(J.ntiles < kNdGrid ? J.ntiles : kNdGrid);
    return J.lattice ? launch_nd_lat<true>(J, g, s) : launch_nd_lat<false>(J, g, s);
}

}  // namespace vt
