// nd_kernels.hip -- the general path: diagrams in any dimension d = 1 .. 6
// (the paper states the method for any dimension, Sec. 3 problem statement),
// with anisotropic voxels and the same keys as the 2D/3D path:
//     Voronoi q,  Laguerre q - w_s,  Johnson-Mehl t_s + sqrt(q) / v,
// q = d0*d0 + T, T = d1*d1, then T + d2*d2, ... over the remaining axes (the
// 2D and 3D forms are its first cases), minimum-image differences for
// periodic boundaries (App. A, eq. dL), each operation rounded once.
//
// Binning: a counting sort into a uniform d-dimensional bin grid (periodic
// coordinates brought into the unit cell first).
//
// Labelling: one workgroup of 256 threads per tile of at most 256 voxels
// (powers of two per axis), one voxel per thread.
//   1. Rings of bins around the tile are visited until every site beyond them
//      provably loses: UB = the smallest upper bound of a visited site's key
//      over the tile's box of voxel centres, and the sites outside the visited
//      box are at least `gap` away along some axis, so their keys exceed
//      gap^2 (Voronoi), gap^2 - max w (Laguerre), min t + gap / v
//      (Johnson-Mehl).
//   2. The visited sites whose lower bound over the tile is <= UB + M are
//      staged in LDS and every thread takes the lexicographic minimum of
//      (key, site index) over them: the brute-force result with ties to the
//      lowest index, whatever the order of the candidates.
// M = 2^-36 of the key scale, far above the rounding error of any bound or
// key, so a dropped site's computed key is strictly above the winner's.
#include "vt_internal.h"

namespace vt {

namespace {

constexpr int NDT = 256;    // threads per workgroup, one voxel each
constexpr int ND_CAP = 512; // candidates staged in LDS per evaluation round
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

// ------------------------------------------------------------------ binning

__global__ __launch_bounds__(NDT) void k_nd_count(NdDev J)
{
    const int64_t i = blockIdx.x * (int64_t)NDT + threadIdx.x;
    const bool live = i < J.nsites;
    unsigned long long hi = 0ull, lo = 0ull;
    if (live) {
        const int nd = J.ndim;
        bool ok = true;
        int64_t lin = 0, stride = 1;
        for (int a = 0; a < nd; ++a) {
            double c = J.coords[i * nd + a];
            if (J.bc && isfinite(c))
                c = cell_coord(c, J.L[a]);
            int b = 0;
            if (!(c >= 0.0 && c < J.L[a])) {
                ok = false;
            } else {
                const int v = (int)(c * J.inv_bs[a]);
                b = v < 0 ? 0 : (v >= J.nb[a] ? J.nb[a] - 1 : v);
            }
            lin += b * stride;
            stride *= J.nb[a];
        }
        if (J.kind != KIND_VORONOI) {
            const double p = J.param[i];
            if (!isfinite(p)) {
                ok = false;
            } else {
                hi = nd_ordered(p);
                lo = nd_ordered(-p);
            }
        }
        if (!ok) {
            lin = 0;
            hi = lo = 0ull;
            atomicOr(J.status, ST_INPUT);
        }
        J.site_bin[i] = (int32_t)lin;
        J.site_rank[i] = atomicAdd(&J.bin_count[lin], 1);
    }
    if (J.kind == KIND_VORONOI)
        return;
    // parameter bounds: reduce over the wavefront, one atomic per wavefront
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long h2 = __shfl_xor(hi, o), l2 = __shfl_xor(lo, o);
        hi = h2 > hi ? h2 : hi;
        lo = l2 > lo ? l2 : lo;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        if (hi)
            atomicMax(&J.pbound[0], hi);
        if (lo)
            atomicMax(&J.pbound[1], lo);
    }
}

__global__ __launch_bounds__(NDT) void k_nd_scatter(NdDev J)
{
    const int64_t i = blockIdx.x * (int64_t)NDT + threadIdx.x;
    if (i >= J.nsites)
        return;
    const int nd = J.ndim;
    const int64_t pos = J.bin_start[J.site_bin[i]] + J.site_rank[i];
    for (int a = 0; a < nd; ++a) {
        const double c = J.coords[i * nd + a];
        J.sc[pos * nd + a] = J.bc ? cell_coord(c, J.L[a]) : c;
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

struct NdLds {
    double c[kMaxDim][ND_CAP];
    double p[ND_CAP];
    int32_t idx[ND_CAP];
    int32_t count;
    double red[NDT / WAVE];
    int32_t ired[NDT / WAVE];
};

__device__ inline double block_min(double v, NdLds& S)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmin(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0)
        S.red[threadIdx.x / WAVE] = v;
    __syncthreads();
    double r = S.red[0];
    for (int w = 1; w < NDT / WAVE; ++w)
        r = fmin(r, S.red[w]);
    return r;
}

__device__ inline int block_max_int(int v, NdLds& S)
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

// Bounds of the key of the sorted site `pos` over the tile's box of voxel
// centres [lo, hi]: per axis the smallest and largest (minimum-image)
// distance to the box, then the key of the kind.
template <int KIND, int DIM>
__device__ inline void site_bounds(const NdDev& J, const NdConst& C, int64_t pos, const double* lo,
                                   const double* hi, double& kl, double& ku)
{
    const int nd = DIM;
    double lq = 0.0, uq = 0.0;
#pragma unroll
    for (int a = 0; a < nd; ++a) {
        const double s = J.sc[pos * nd + a];
        double dmin, dmax;
        if (!J.bc) {
            dmin = fmax(0.0, fmax(lo[a] - s, s - hi[a]));
            dmax = fmax(fabs(s - lo[a]), fabs(s - hi[a]));
        } else {
            // images s - L, s, s + L cover every voxel centre of the cell
            dmin = __builtin_inf();
            dmax = __builtin_inf();
            for (int k = -1; k <= 1; ++k) {
                const double sk = s + (double)k * J.L[a];
                dmin = fmin(dmin, fmax(0.0, fmax(lo[a] - sk, sk - hi[a])));
                dmax = fmin(dmax, fmax(fabs(sk - lo[a]), fabs(sk - hi[a])));
            }
            dmax = fmin(dmax, J.H[a]);
        }
        lq += dmin * dmin;
        uq += dmax * dmax;
    }
    const double p = J.sp[pos];
    if (KIND == KIND_VORONOI) {
        kl = lq;
        ku = uq;
    } else if (KIND == KIND_LAGUERRE) {
        kl = lq - p;
        ku = uq - p;
    } else {
        kl = p + sqrt(lq) * C.rv;
        ku = p + sqrt(uq) * C.rv;
    }
}

// The visited bin box of ring r around the tile's bins [bl, bh]: per axis the
// first bin (unwrapped) and the width; full = the axis is covered entirely.
struct NdBox {
    int first[kMaxDim], width[kMaxDim];
    bool full[kMaxDim];
    int64_t count;
};

template <int DIM>
__device__ inline NdBox ring_box(const NdDev& J, const int* bl, const int* bh, int r)
{
    NdBox B;
    B.count = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int f = bl[a] - r, e = bh[a] + r;
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

// Smallest distance from the tile's box to a site outside the visited box
// (infinite once every site has been visited).
template <int DIM>
__device__ inline double outside_gap(const NdDev& J, const NdBox& B, const double* lo, const double* hi)
{
    double g = __builtin_inf();
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (J.bc) {
            if (B.full[a])
                continue;
            const double low = lo[a] - (double)B.first[a] * J.bs[a];
            const double high = (double)(B.first[a] + B.width[a]) * J.bs[a] - hi[a];
            g = fmin(g, fmin(low, high));
        } else {
            if (B.first[a] > 0)
                g = fmin(g, lo[a] - (double)B.first[a] * J.bs[a]);
            if (B.first[a] + B.width[a] < J.nb[a])
                g = fmin(g, (double)(B.first[a] + B.width[a]) * J.bs[a] - hi[a]);
        }
    }
    return fmax(g, 0.0);
}

// The exact key of a staged candidate at voxel centre x (same operations as
// the problem's definition; see the file comment).
template <int KIND, int DIM>
__device__ inline double nd_key(const NdDev& J, const NdLds& S, int k, const double* x)
{
    const int nd = DIM;
    double d = S.c[0][k] - x[0];
    if (J.bc)
        d = d >= J.H[0] ? d - J.L[0] : (d < -J.H[0] ? d + J.L[0] : d);
    double q = d * d;
    if (nd > 1) {
        double e = S.c[1][k] - x[1];
        if (J.bc)
            e = e >= J.H[1] ? e - J.L[1] : (e < -J.H[1] ? e + J.L[1] : e);
        double T = e * e;
#pragma unroll
        for (int a = 2; a < nd; ++a) {
            double f = S.c[a][k] - x[a];
            if (J.bc)
                f = f >= J.H[a] ? f - J.L[a] : (f < -J.H[a] ? f + J.L[a] : f);
            T = T + f * f;
        }
        q = q + T;
    }
    const double p = S.p[k];
    if (KIND == KIND_VORONOI)
        return q;
    if (KIND == KIND_LAGUERRE)
        return q - p;
    return J.jm_div ? p + key_sqrt(q) / J.growth : p + key_sqrt(q) * J.rgrowth;
}

template <int KIND, int DIM>
__device__ inline void nd_evaluate(const NdDev& J, const NdLds& S, int count, const double* x, double& best,
                                   int& blab)
{
    for (int k = 0; k < count; ++k) {
        const double key = nd_key<KIND, DIM>(J, S, k, x);
        const int id = S.idx[k];
        if (key < best || (key == best && id < blab)) {
            best = key;
            blab = id;
        }
    }
}

template <int KIND, int DIM>
__global__ __launch_bounds__(NDT) void k_nd_label(NdDev J)
{
    __shared__ NdLds S;
    const int tid = threadIdx.x;
    const int nd = DIM;
    const bool bad = *(volatile int32_t*)J.status != 0;
    NdConst C;
    {
        double sumL2 = 0.0;
        for (int a = 0; a < nd; ++a)
            sumL2 += J.L[a] * J.L[a];
        C.rv = J.rgrowth;
        C.pmax = C.pmin = 0.0;
        if (KIND != KIND_VORONOI && !bad) {
            C.pmax = nd_from_ordered(J.pbound[0]);
            C.pmin = -nd_from_ordered(J.pbound[1]);
        }
        const double pabs = fmax(fabs(C.pmax), fabs(C.pmin));
        const double scale = KIND == KIND_VORONOI ? sumL2
                           : KIND == KIND_LAGUERRE ? sumL2 + 2.0 * pabs
                                                   : sqrt(sumL2) * C.rv + 2.0 * pabs;
        C.M = scale * 0x1p-36;
    }
    for (int64_t t = blockIdx.x; t < J.ntiles; t += gridDim.x) {
        // the tile: voxels [v0, ve] per axis; centres [lo, hi]
        int64_t v0[kMaxDim], ve[kMaxDim], vi[kMaxDim];
        double lo[kMaxDim], hi[kMaxDim], x[kMaxDim];
        int bl[kMaxDim], bh[kMaxDim];
        int64_t rem = t;
        int l = tid;
        bool live = true;
#pragma unroll
        for (int a = 0; a < nd; ++a) {
            const int64_t tc = rem % J.nt[a];
            rem /= J.nt[a];
            v0[a] = tc * J.T[a];
            ve[a] = (v0[a] + J.T[a] < J.n[a] ? v0[a] + J.T[a] : J.n[a]) - 1;
            lo[a] = ((double)v0[a] + 0.5) * J.h[a];
            hi[a] = ((double)ve[a] + 0.5) * J.h[a];
            const int off = l % J.T[a];
            l /= J.T[a];
            vi[a] = v0[a] + off;
            live = live && vi[a] <= ve[a];
            x[a] = ((double)vi[a] + 0.5) * J.h[a];
            const int b0 = (int)(lo[a] * J.inv_bs[a]), b1 = (int)(hi[a] * J.inv_bs[a]);
            bl[a] = min(max(b0, 0), J.nb[a] - 1);
            bh[a] = min(max(b1, 0), J.nb[a] - 1);
        }
        live = live && l == 0;
        double best = __builtin_inf();
        int blab = 0x7fffffff;
        if (!bad) {
            // 1. rings of bins until the sites beyond them provably lose
            double UB = __builtin_inf();
            int r = 0;
            NdBox B = ring_box<DIM>(J, bl, bh, 0), P = B;
            for (;;) {
                double my = __builtin_inf();
                for (int64_t j = tid; j < B.count; j += NDT) {
                    bool in_prev;
                    const int64_t lin = box_bin<DIM>(J, B, j, P, r > 0, in_prev);
                    if (in_prev)
                        continue;
                    const int s1 = J.bin_start[lin + 1];
                    for (int s = J.bin_start[lin]; s < s1; ++s) {
                        double kl, ku;
                        site_bounds<KIND, DIM>(J, C, s, lo, hi, kl, ku);
                        my = fmin(my, ku);
                    }
                }
                UB = fmin(UB, block_min(my, S));
                const double g = outside_gap<DIM>(J, B, lo, hi);
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
            // 2. stage the candidates and take the lexicographic minimum
            if (tid == 0)
                S.count = 0;
            __syncthreads();
            const double cut = UB + C.M;
            for (int64_t base = 0; base < B.count; base += NDT) {
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
                        double kl, ku;
                        site_bounds<KIND, DIM>(J, C, s, lo, hi, kl, ku);
                        if (kl <= cut) {
                            const int slot = atomicAdd(&S.count, 1);
#pragma unroll
                            for (int a = 0; a < nd; ++a)
                                S.c[a][slot] = J.sc[(int64_t)s * nd + a];
                            S.p[slot] = J.sp[s];
                            S.idx[slot] = J.sidx[s];
                        }
                    }
                    __syncthreads();
                    const int cnt = S.count;
                    __syncthreads();  // every thread has read the count before the next appends
                    if (cnt > ND_CAP - NDT) {
                        if (live)
                            nd_evaluate<KIND, DIM>(J, S, cnt, x, best, blab);
                        __syncthreads();
                        if (tid == 0)
                            S.count = 0;
                        __syncthreads();
                    }
                }
            }
            const int cnt = S.count;
            if (live && cnt > 0)
                nd_evaluate<KIND, DIM>(J, S, cnt, x, best, blab);
            __syncthreads();
        }
        if (live) {
            int64_t lin = 0, stride = 1;
#pragma unroll
            for (int a = 0; a < nd; ++a) {
                lin += vi[a] * stride;
                stride *= J.n[a];
            }
            J.labels[lin] = bad ? -1 : blab;
            if (J.keys)
                J.keys[lin] = bad ? __builtin_nan("") : best;
        }
    }
}

}  // namespace

hipError_t launch_nd_bin_count(const NdDev& J, hipStream_t s)
{
    const int64_t g = (J.nsites + NDT - 1) / NDT;
    k_nd_count<<<(unsigned)g, NDT, 0, s>>>(J);
    return hipGetLastError();
}

hipError_t launch_nd_bin_scatter(const NdDev& J, hipStream_t s)
{
    const int64_t g = (J.nsites + NDT - 1) / NDT;
    k_nd_scatter<<<(unsigned)g, NDT, 0, s>>>(J);
    return hipGetLastError();
}

namespace {

template <int DIM>
void launch_nd_dim(const NdDev& J, unsigned g, hipStream_t s)
{
    if (J.kind == KIND_VORONOI)
        k_nd_label<KIND_VORONOI, DIM><<<g, NDT, 0, s>>>(J);
    else if (J.kind == KIND_LAGUERRE)
        k_nd_label<KIND_LAGUERRE, DIM><<<g, NDT, 0, s>>>(J);
    else
        k_nd_label<KIND_JM, DIM><<<g, NDT, 0, s>>>(J);
}

}  // namespace

hipError_t launch_nd_label(const NdDev& J, hipStream_t s)
{
    const unsigned g = (unsigned)(J.ntiles < kNdGrid ? J.ntiles : kNdGrid);
    switch (J.ndim) {
    case 1: launch_nd_dim<1>(J, g, s); break;
    case 2: launch_nd_dim<2>(J, g, s); break;
    case 3: launch_nd_dim<3>(J, g, s); break;
    case 4: launch_nd_dim<4>(J, g, s); break;
    case 5: launch_nd_dim<5>(J, g, s); break;
    case 6: launch_nd_dim<6>(J, g, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace vt
