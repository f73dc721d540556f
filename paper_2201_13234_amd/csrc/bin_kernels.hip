// bin_kernels.hip -- site binning on the device: a counting sort of the
// sites into a uniform grid of bins (count with atomics, exclusive prefix
// scan of the counts, scatter).  The labelling kernel then finds the sites
// near a voxel tile by walking bins outward from it.
//
// One thread per site.  In a batch, a thread finds its job by binary search
// over the per-job site offsets.  The count pass also checks every site
// (finite coordinates, inside [0, L_a) unless the boundaries are periodic;
// finite parameter; problem statement of Sec. 3) and records max(param) and
// max(-param) for the labelling kernel's lower bounds.  Periodic coordinates
// are brought into the unit cell (cell_coord) by both passes, so the sorted
// sites always lie in [0, L_a).
#include "bin_internal.h"

#include <cstring>

namespace vt {

namespace {

constexpr int kBlock = 256;

__device__ inline unsigned long long ordered_bits(double v)
{
    // Monotone map from binary64 to uint64 (larger double -> larger integer).
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ inline int find_segment(const int64_t* prefix, int n, int64_t g)
{
    // Largest j in [0, n) with prefix[j] <= g.
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

// The counting pass proper: thread g counts site g (of the batch enumeration)
// into its bin.  Invalid sites are ORed into status_acc when it is given,
// else into their job's status word.
__device__ inline void count_sites(const JobDev& single, const JobDev* __restrict__ jobs, int njobs,
                                   const int64_t* __restrict__ prefix, int64_t total, int32_t* status_acc)
{
    const int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const bool live = g < total;
    int j = 0;
    int64_t i = g;
    if (jobs && live) {
        j = find_segment(prefix, njobs, g);
        i = g - prefix[j];
    }
    unsigned long long hi = 0ull, lo = 0ull;  // ordered bits of param and -param, 0 = none
    bool weighted = false;
    if (live) {
        const JobDev& J = jobs ? jobs[j] : single;
        const int nd = J.ndim;
        weighted = J.kind != KIND_VORONOI;
        bool ok = true;
        int b[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
            if (a < nd) {
                double c = J.coords[i * nd + a];
                if (J.bc && isfinite(c))
                    c = cell_coord(c, J.L[a]);
                if (!(c >= 0.0 && c < J.L[a])) {
                    ok = false;
                } else {
                    int v = (int)(c * J.inv_bs[a]);  // c >= 0: truncation is floor
                    b[a] = v < 0 ? 0 : (v >= J.nb[a] ? J.nb[a] - 1 : v);
                }
            }
        }
        double p = 0.0;
        if (weighted) {
            p = J.param[i];
            if (!(fabs(p) <= VT_SCALE_MAX))  // also false for NaN
                ok = false;
        }
        if (!ok) {
            b[0] = b[1] = b[2] = 0;
            atomicOr(status_acc ? status_acc : J.status, ST_INPUT);
        }
        int lin = b[0] + J.nb[0] * (b[1] + J.nb[1] * b[2]);
        int rank = atomicAdd(&J.bin_count[lin], 1);
        J.site_bin[i] = lin;
        J.site_rank[i] = rank;
        if (weighted && ok) {
            hi = ordered_bits(p);
            lo = ordered_bits(-p);
        }
    }
    // Parameter bounds.  A wavefront whose live lanes belong to one job reduces
    // over its lanes (dead lanes carry 0); a block whose wavefronts all do so
    // for the same job reduces once more through LDS and issues one atomic per
    // bound, so that the atomics on the two shared addresses stay few.
    // Otherwise the wavefront's first lane, or each site of a mixed
    // wavefront, issues its own.  Live lanes are a prefix of the grid, so lane
    // 0 of a wavefront (thread 0 of a block) is live if any lane is.
    __shared__ int bjob[kBlock / WAVE];
    __shared__ unsigned long long bhi[kBlock / WAVE], blo[kBlock / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int j0 = __shfl(j, 0);
    const bool wuni = __all(!live || j == j0);
    if (wuni) {
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long h2 = __shfl_xor(hi, o), l2 = __shfl_xor(lo, o);
            hi = h2 > hi ? h2 : hi;
            lo = l2 > lo ? l2 : lo;
        }
    }
    if (lane == 0) {
        bjob[w] = !wuni ? -2 : (live ? j0 : -1);
        bhi[w] = hi;
        blo[w] = lo;
    }
    __syncthreads();
    int jb = -1;
    bool buni = true;
    for (int k = 0; k < kBlock / WAVE; ++k) {
        const int v = bjob[k];
        if (v == -2 || (v >= 0 && jb >= 0 && v != jb))
            buni = false;
        if (v >= 0)
            jb = v;
    }
    if (buni) {
        if (threadIdx.x == 0 && jb >= 0 && weighted) {
            for (int k = 1; k < kBlock / WAVE; ++k) {
                hi = bhi[k] > hi ? bhi[k] : hi;
                lo = blo[k] > lo ? blo[k] : lo;
            }
            const JobDev& J = jobs ? jobs[jb] : single;
            if (hi)
                atomicMax(&J.pbound[0], hi);
            if (lo)
                atomicMax(&J.pbound[1], lo);
        }
        return;
    }
    if (!live || (wuni && lane != 0))
        return;
    if (weighted) {
        const JobDev& J = jobs ? jobs[j] : single;
        if (hi)
            atomicMax(&J.pbound[0], hi);
        if (lo)
            atomicMax(&J.pbound[1], lo);
    }
}

// With status_acc given (one job), thread 0 also publishes the status the
// count accumulated there: the labelling kernels read it from *J.status.
__global__ __launch_bounds__(kBlock) void k_bin_scatter(JobDev single, const JobDev* __restrict__ jobs,
                                                        int njobs, const int64_t* __restrict__ prefix,
                                                        int64_t total, const int32_t* __restrict__ status_acc)
{
    int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (g >= total)
        return;
    int j = 0;
    int64_t i = g;
    if (jobs) {
        j = find_segment(prefix, njobs, g);
        i = g - prefix[j];
    }
    const JobDev& J = jobs ? jobs[j] : single;
    if (status_acc && g == 0)
        *J.status = *status_acc;
    const int nd = J.ndim;
    int lin = J.site_bin[i];
    int pos = J.bin_start[lin] + J.site_rank[i];
    const double* c = J.coords + i * nd;
    double4 rec;
    rec.x = J.bc ? cell_coord(c[0], J.L[0]) : c[0];
    rec.y = J.bc ? cell_coord(c[1], J.L[1]) : c[1];
    rec.z = nd == 3 ? (J.bc ? cell_coord(c[2], J.L[2]) : c[2]) : 0.0;
    rec.w = J.kind != KIND_VORONOI ? J.param[i] : 0.0;
    J.sites[pos] = rec;
    J.sidx[pos] = (int32_t)i;
}

// ---- Johnson-Mehl: sites that never win ----
//
// A site s never wins, nor ties, at any voxel if another site r satisfies
// t_r + d(r, s) / v < t_s - M: by the triangle inequality (which the periodic
// distance obeys too) t_r + d(x, r) / v <= t_r + d(r, s) / v + d(x, s) / v <
// t_s + d(x, s) / v - M for every x, and M (2^-36 of the key scale) is far
// above the rounding error of any computed key.  The paper notes that such
// nucleation sites are ineffective (Sec. 3.3); dropping them from the bins leaves
// the labels unchanged and shortens every candidate list.  A swallowing site
// lies within (t_s - min t) * v of s, so the search only visits bins that
// close; a site whose search box exceeds kPruneMaxBins bins is kept.

constexpr int kPruneMaxBins = 4096;
// Lanes per site of a single job's search (WAVE / kJmLanes sites per wavefront).
constexpr int kJmLanes = 16;

__device__ inline double from_ordered_bits(unsigned long long u)
{
    unsigned long long b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)b);
}

__device__ inline int find_bin_job(const JobDev* jobs, int n, int64_t g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].bin_begin <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Whether another site swallows the site at sorted position g (see above),
// for a group of GL lanes of the wavefront (WAVE / GL sites per wavefront;
// lane lig of group grp; valid false for a group past the last site).  The
// group's lanes take the bins of the search box, GL at a time, and each lane
// reads its bin's sites two at a time so that their loads are in flight
// together (bins hold about one site at the Johnson-Mehl bin size).  The test
// compares squares, (d / v)^2 < (t_s - M - t_r)^2 with t_s - M - t_r > 0: its
// rounding, a few units in the last place of the key scale, is as far below M
// as that of the key itself.  Every lane of the wavefront calls this (the
// loop's ballots are wavefront-wide).
template <int ND, int GL>
__device__ inline bool jm_swallowed(const JobDev& J, int64_t g, bool valid, int lig, int grp)
{
    const double4 s = valid ? J.sites[g] : make_double4(0.0, 0.0, 0.0, 0.0);
    const double sc[3] = {s.x, s.y, s.z};
    const double tmin = -from_ordered_bits(J.pbound[1]), tmax = from_ordered_bits(J.pbound[0]);
    double sumL2 = 0.0;
#pragma unroll
    for (int a = 0; a < ND; ++a)
        sumL2 += J.L[a] * J.L[a];
    const double M = (sqrt(sumL2) * J.rgrowth + 2.0 * fmax(fabs(tmin), fabs(tmax))) * 0x1p-36;
    const bool periodic = J.bc != 0;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < ND; ++a)
        inside = inside && sc[a] >= 0.0 && sc[a] < J.L[a];  // invalid input (reported by the count kernel): keep
    const double tcut = s.w - M;
    const double gap = tcut - tmin;
    bool active = valid && inside && gap > 0.0;
    int lo[3] = {0, 0, 0}, cnt3[3] = {1, 1, 1};
    int nbox = 0;
    if (active) {
        const double R = gap * J.growth * (1.0 + 0x1p-20) + J.L[0] * 0x1p-30;
        int64_t nb64 = 1;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            const int nb = J.nb[a];
            const double l = floor((sc[a] - R) * J.inv_bs[a]), h = floor((sc[a] + R) * J.inv_bs[a]);
            int la, ha;
            if (!(h - l + 1.0 < (double)nb)) {  // the whole axis (also catches a huge R)
                la = 0;
                ha = nb - 1;
            } else if (periodic) {
                la = (int)l;  // in (-nb, 2 nb): wrapped below
                ha = (int)h;
            } else {
                la = max((int)l, 0);
                ha = min((int)h, nb - 1);
            }
            lo[a] = la;
            cnt3[a] = ha - la + 1;
            nb64 *= cnt3[a];
        }
        active = nb64 <= kPruneMaxBins;
        nbox = active ? (int)nb64 : 0;
    }
    const double rg2 = J.rgrowth * J.rgrowth;
    double Lh[3], La[3];
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        La[a] = J.L[a];
        Lh[a] = 0.5 * J.L[a];
    }
    const int nx = cnt3[0], nxy = cnt3[0] * cnt3[1];
    bool found = false;
    for (int e0 = 0;; e0 += GL) {
        const bool act = active && !found && e0 < nbox;
        if (__ballot(act) == 0)
            break;
        const int e = e0 + lig;
        bool hit = false;
        if (act && e < nbox) {
            const int ez = e / nxy, rem = e - ez * nxy, ey = rem / nx, ex = rem - ey * nx;
            const int bb[3] = {lo[0] + ex, lo[1] + ey, lo[2] + ez};
            int w3[3] = {0, 0, 0};
#pragma unroll
            for (int a = 0; a < ND; ++a) {
                const int nb = J.nb[a];
                w3[a] = bb[a] < 0 ? bb[a] + nb : (bb[a] >= nb ? bb[a] - nb : bb[a]);
            }
            const int lin = w3[0] + J.nb[0] * (w3[1] + J.nb[1] * w3[2]);
            const int b0 = J.bin_start[lin], cnt = J.bin_count[lin];
            for (int k = 0; k < cnt && !hit; k += 2) {
                double4 q[2];
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    q[u] = k + u < cnt ? J.sites[b0 + k + u] : s;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const double qc[3] = {q[u].x, q[u].y, q[u].z};
                    double d2 = 0.0;
#pragma unroll
                    for (int a = 0; a < ND; ++a) {
                        double d = sc[a] - qc[a];
                        if (periodic)
                            d = d >= Lh[a] ? d - La[a] : (d < -Lh[a] ? d + La[a] : d);
                        d2 += d * d;
                    }
                    const double rhs = tcut - q[u].w;
                    const bool other = k + u < cnt && (int64_t)b0 + k + u != g;
                    hit = hit || (other && rhs > 0.0 && d2 * rg2 < rhs * rhs);
                }
            }
        }
        const unsigned long long b = __ballot(hit);
        if constexpr (GL == WAVE)
            found = found || b != 0;
        else
            found = found || ((b >> (grp * GL)) & ((1ull << GL) - 1)) != 0;
    }
    return found;
}

// Marks (in site_bin, indexed by the job's sorted position) the sites that
// some other site swallows: WAVE / GL sites per wavefront, GL lanes each.
// Batches take one site per wavefront (GL = WAVE), so that a wavefront's
// sites belong to one job and its record sits in scalar registers, copied
// once, and the search loops read none of its fields through memory.
template <int GL>
__global__ __launch_bounds__(kBlock) void k_jm_mark(JobDev single, const JobDev* __restrict__ jobs, int njobs,
                                                    const int64_t* __restrict__ prefix, int64_t total)
{
    constexpr int kSites = WAVE / GL;
    const int lane = threadIdx.x & (WAVE - 1), grp = lane / GL, lig = lane % GL;
    const int64_t w = blockIdx.x * (int64_t)(kBlock / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int64_t g0 = w * kSites;
    if (g0 >= total)
        return;
    const int64_t g = g0 + grp;
    const bool valid = g < total;
    if constexpr (GL == WAVE) {
        if (jobs) {
            const int j = __builtin_amdgcn_readfirstlane(find_segment(prefix, njobs, g));
            const JobDev J = jobs[j];
            if (J.kind != KIND_JM)
                return;
            const bool dead = J.ndim == 3 ? jm_swallowed<3, GL>(J, g, valid, lig, grp)
                                          : jm_swallowed<2, GL>(J, g, valid, lig, grp);
            if (lig == 0)
                J.site_bin[g - J.site_begin] = dead ? 1 : 0;
            return;
        }
    }
    if (single.kind != KIND_JM)
        return;
    const bool dead = single.ndim == 3 ? jm_swallowed<3, GL>(single, g, valid, lig, grp)
                                       : jm_swallowed<2, GL>(single, g, valid, lig, grp);
    if (valid && lig == 0)
        single.site_bin[g - single.site_begin] = dead ? 1 : 0;
}

// Moves the live sites of each bin to the front of its range and stores their
// number in bin_count.
__global__ __launch_bounds__(kBlock) void k_jm_compact(JobDev single, const JobDev* __restrict__ jobs, int njobs,
                                                       int64_t total_bins)
{
    const int64_t gb = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (gb >= total_bins)
        return;
    const int j = jobs ? find_bin_job(jobs, njobs, gb) : 0;
    const JobDev& J = jobs ? jobs[j] : single;
    if (J.kind != KIND_JM)
        return;
    const int64_t b = gb - J.bin_begin;
    const int b0 = J.bin_start[b], cnt = J.bin_count[b];
    int w = 0;
    for (int k = 0; k < cnt; ++k) {
        const int r = b0 + k;
        if (J.site_bin[r - J.site_begin] != 0)
            continue;
        if (w != k) {
            J.sites[b0 + w] = J.sites[r];
            J.sidx[b0 + w] = J.sidx[r];
        }
        ++w;
    }
    J.bin_count[b] = w;
}

// ---- exclusive prefix scan of int32 counts: reduce, scan partials, final ----

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int wave_inclusive_add(int v, int lane)
{
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(v, o);
        if (lane >= o)
            v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over the block; returns the
// exclusive prefix and the block total.
__device__ inline int block_exclusive_add(int v, int& total)
{
    __shared__ int wsum[kScanThreads / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    int inc = wave_inclusive_add(v, lane);
    if (lane == WAVE - 1)
        wsum[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
    for (int k = 0; k < kScanThreads / WAVE; ++k) {
        int s = wsum[k];
        if (k < w)
            off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

// Exclusive scan out[0..n] of cnt[0..n) (n <= kSmallScanMax) by one
// workgroup of at most 16 wavefronts: wavefront w takes ROWS consecutive rows
// of 256 counts, each lane four adjacent counts of a row, so that every load
// moves 1 KiB of contiguous words.  cnt must be padded with zeros to whole
// wavefronts (count_words) and out sized for as many words plus one: whole
// rows are written.  The code is straight-line: all loads are issued before
// the first is used, and the row scans before the first store.
template <int ROWS>
__global__ __launch_bounds__(1024) void k_scan_small(const int32_t* __restrict__ cnt, int32_t* __restrict__ out,
                                                     int n)
{
    __shared__ int wtot[1024 / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    const int seg = w * ROWS * 256;
    int4 v[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
        v[r] = *(const int4*)(cnt + seg + r * 256 + lane * 4);
    int inc[ROWS];
    int lsum = 0;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int s4 = (v[r].x + v[r].y) + (v[r].z + v[r].w);
        inc[r] = wave_inclusive_add(s4, lane);
        lsum += s4;
    }
    for (int o = 32; o > 0; o >>= 1)
        lsum += __shfl_xor(lsum, o);
    if (lane == 0)
        wtot[w] = lsum;
    __syncthreads();
    int carry = 0, grand = 0;
    for (int k = 0; k < nw; ++k) {
        carry += k < w ? wtot[k] : 0;
        grand += wtot[k];
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int s4 = (v[r].x + v[r].y) + (v[r].z + v[r].w);
        const int e0 = carry + inc[r] - s4, e1 = e0 + v[r].x, e2 = e1 + v[r].y, e3 = e2 + v[r].z;
        *(int4*)(out + seg + r * 256 + lane * 4) = make_int4(e0, e1, e2, e3);
        carry += __builtin_amdgcn_readlane(inc[r], WAVE - 1);
    }
    // out[n], the total, is the row value at index n unless the rows end there
    if (n == nw * ROWS * 256 && threadIdx.x == 0)
        out[n] = grand;
}

// The counting kernel.  For one job it can also store the job's record and
// clear the next call's zeroed scratch (see CountTail).  Batches pass an empty
// tail.
__global__ __launch_bounds__(kBlock) void k_bin_count(JobDev single, const JobDev* __restrict__ jobs, int njobs,
                                                      const int64_t* __restrict__ prefix, int64_t total,
                                                      CountTail tail)
{
    if (tail.clear) {
        const int64_t stride = (int64_t)gridDim.x * kBlock, nq = tail.clear_words / 4;
        int4* q = (int4*)tail.clear;
        for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nq; k += stride)
            q[k] = make_int4(0, 0, 0, 0);
    }
    if (tail.job_dst && blockIdx.x == 0 && threadIdx.x == 0)
        *tail.job_dst = single;
    count_sites(single, jobs, njobs, prefix, total, tail.status_acc);
}

// One-pass exclusive scan of the bin counts (a chained scan with decoupled
// look-back: Merrill and Garland, Single-pass Parallel Prefix Scan with
// Decoupled Look-back, 2016).  Each workgroup scans one tile of kScanTile
// counts and publishes, in its flag word, first the tile total and then its
// inclusive prefix; it finds its own exclusive prefix by walking back over
// the flags of the tiles before it, adding totals until it meets a published
// prefix.  A flag word is 0 (nothing yet), kAggr | total or kIncl | prefix
// (values below 2^31); the flags start at zero (the caller clears them).
// Workgroups wait only on tiles of lower index, which were dispatched before
// them.  One launch instead of reduce, scan-of-partials and final passes.
constexpr unsigned long long kAggr = 1ull << 62, kIncl = 2ull << 62, kValMask = (1ull << 62) - 1;

__global__ __launch_bounds__(kScanThreads) void k_scan_onepass(const int32_t* __restrict__ in,
                                                               int32_t* __restrict__ out, int64_t n,
                                                               unsigned long long* __restrict__ flags)
{
    __shared__ int prefix_sh;
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        sum += v[k];
    }
    int total;
    const int ex = block_exclusive_add(sum, total);
    if (threadIdx.x == 0) {
        int before = 0;
        if (tile == 0) {
            __hip_atomic_store(&flags[0], kIncl | (unsigned long long)total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&flags[tile], kAggr | (unsigned long long)total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            for (int64_t k = tile - 1; k >= 0;) {
                const unsigned long long f = __hip_atomic_load(&flags[k], __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                if (f == 0ull) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                before += (int)(f & kValMask);
                if ((f & ~kValMask) == kIncl)
                    break;
                --k;
            }
            __hip_atomic_store(&flags[tile], kIncl | (unsigned long long)(before + total), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        prefix_sh = before;
    }
    __syncthreads();
    int run = prefix_sh + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n)
            out[base + k] = run;
        if (base + k == n - 1)
            out[n] = run + v[k];
        run += v[k];
    }
}

inline unsigned grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    unsigned g = grid_for(n, 256);
    if (g > 4096)
        g = 4096;
    k_fill_i32<<<g, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    unsigned g = grid_for(n, 256);
    if (g > 4096)
        g = 4096;
    k_fill_u64<<<g, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_bin_count(const JobDev& single, const JobDev* jobs_dev, int njobs,
                            const int64_t* site_prefix_dev, int64_t total_sites, hipStream_t s)
{
    if (total_sites <= 0)
        return hipSuccess;
    CountTail none;
    std::memset(&none, 0, sizeof none);
    k_bin_count<<<grid_for(total_sites, kBlock), kBlock, 0, s>>>(single, jobs_dev, njobs, site_prefix_dev,
                                                                total_sites, none);
    return hipGetLastError();
}

hipError_t launch_bin_count_single(const JobDev& job, const CountTail& tail, hipStream_t s)
{
    if (job.nsites <= 0 || (tail.clear_words & 3) != 0 || ((uintptr_t)tail.clear & 15) != 0)
        return hipErrorInvalidValue;
    k_bin_count<<<grid_for(job.nsites, kBlock), kBlock, 0, s>>>(job, nullptr, 1, nullptr, job.nsites, tail);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const JobDev& single, const JobDev* jobs_dev, int njobs,
                              const int64_t* site_prefix_dev, int64_t total_sites, hipStream_t s)
{
    if (total_sites <= 0)
        return hipSuccess;
    k_bin_scatter<<<grid_for(total_sites, kBlock), kBlock, 0, s>>>(single, jobs_dev, njobs,
                                                                  site_prefix_dev, total_sites, nullptr);
    return hipGetLastError();
}

hipError_t launch_scan_small(const int32_t* cnt, int32_t* out, int64_t n, hipStream_t s)
{
    if (n <= 0 || n > kSmallScanMax || ((uintptr_t)cnt & 15) != 0 || ((uintptr_t)out & 15) != 0)
        return hipErrorInvalidValue;
    const int64_t per_wave = small_scan_wave_counts(n);
    const unsigned threads = (unsigned)((n + per_wave - 1) / per_wave) * WAVE;
    if (per_wave == 8 * 256)
        k_scan_small<8><<<1, threads, 0, s>>>(cnt, out, (int)n);
    else
        k_scan_small<16><<<1, threads, 0, s>>>(cnt, out, (int)n);
    return hipGetLastError();
}

hipError_t launch_bin_scatter_single(const JobDev& job, const int32_t* status_acc, hipStream_t s)
{
    if (job.nsites <= 0)
        return hipErrorInvalidValue;
    k_bin_scatter<<<grid_for(job.nsites, kBlock), kBlock, 0, s>>>(job, nullptr, 1, nullptr, job.nsites,
                                                                 status_acc);
    return hipGetLastError();
}

hipError_t launch_jm_prune(const JobDev& single, const JobDev* jobs_dev, int njobs,
                           const int64_t* site_prefix_dev, int64_t total_sites, int64_t total_bins, hipStream_t s)
{
    if (total_sites <= 0 || total_bins <= 0)
        return hipSuccess;
    if (jobs_dev) {
        k_jm_mark<WAVE><<<grid_for(total_sites, kBlock / WAVE), kBlock, 0, s>>>(single, jobs_dev, njobs,
                                                                           site_prefix_dev, total_sites);
    } else {
        constexpr int kSites = WAVE / kJmLanes;  // sites per wavefront
        k_jm_mark<kJmLanes><<<grid_for(total_sites, kBlock / WAVE * kSites), kBlock, 0, s>>>(
            single, nullptr, 1, nullptr, total_sites);
    }
    k_jm_compact<<<grid_for(total_bins, kBlock), kBlock, 0, s>>>(single, jobs_dev, njobs, total_bins);
    return hipGetLastError();
}

int64_t scan_flags_needed(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, unsigned long long* flags,
                       int64_t flags_cap, hipStream_t s)
{
    int64_t nblk = (n + kScanTile - 1) / kScanTile;
    if (n <= 0 || nblk > flags_cap || nblk > 0x7fffffff)
        return hipErrorInvalidValue;
    k_scan_onepass<<<(unsigned)nblk, kScanThreads, 0, s>>>(in, out, n, flags);
    return hipGetLastError();
}

}  // namespace vt
