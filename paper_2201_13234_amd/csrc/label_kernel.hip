// label_kernel.hip -- per-voxel argmin of the diagram's key over the sites.
//
// What is computed (Sec. 2, Sec. 3 problem statement, App. A): for every voxel
// centre x, the lowest index s minimising
//     Voronoi q,  Laguerre q - w_s,  Johnson-Mehl t_s + sqrt(q) / v,
// q = d0*d0 + (d1*d1 + d2*d2) with minimum-image differences for periodic
// boundaries, each operation rounded once in binary64 (the build keeps the
// compiler from contracting into fused multiply-add).
//
// How (our GPU design, not the paper's CPU ball scheme):
//   A workgroup of four wavefronts owns a region of four voxel tiles.
//   1. Region gather (whole workgroup).  The bins around the region are loaded
//      into LDS, many per round.  Every site gets an upper bound of its key
//      over the region's box of voxel centres; UB = the smallest of them bounds
//      the winning key of every voxel of the region.  A face of the visited
//      bin box is moved outward until the sites beyond it provably lose:
//      gap^2 > UB (Voronoi), gap^2 - max w > UB (Laguerre),
//      min t + gap / v > UB (Johnson-Mehl).
//   2. Tile pruning (one wavefront per tile).  Sites whose lower bound over the
//      tile exceeds the tile's own UB are dropped, then every site that another
//      site beats on the whole tile: the key difference of two sites is linear
//      in x for Voronoi and Laguerre, so its minimum over the box is at a
//      corner; for Johnson-Mehl a bound of the difference of distances is used.
//   3. Exact evaluation.  The survivors, sorted by site index, are evaluated
//      at every voxel of the lane's run with the exact key and a strict '<':
//      the paper's brute-force loop restricted to the survivors, which keeps
//      the lowest index on ties.
// Every bound test keeps a margin of 2^-36 times the problem's key scale, far
// above the rounding error of any computed key, so a dropped site's computed
// key is strictly larger than the winner's at every voxel: the labels equal
// brute force bit for bit.  A region whose sites do not fit in LDS falls back
// to a per-tile walk that evaluates its candidates in batches.
#include "label_core.h"

namespace vt {

namespace {

template <int KIND, int DIM, int CFG>
__global__ __launch_bounds__(NT) void k_label_single(const JobDev* __restrict__ jp)
{
    __shared__ Smem sm;
    const JobDev& J = job_ref(jp, 0);
    const int64_t r = xcd_unit(blockIdx.x, gridDim.x);
    region_cfg<KIND, DIM, CFG>(J, r, r, sm, threadIdx.x);
}

// What the main kernel left over: first the regions it queued whole (their
// gather overflowed the region list; one workgroup each, with the dense-capable
// gather), then the tiles whose candidate list overflowed (one wavefront each).
template <int KIND, int DIM, int CFG>
__global__ __launch_bounds__(NT) void k_label_fallback(const JobDev* __restrict__ jp)
{
    __shared__ Smem sm;
    __shared__ FallbackLds fb[NW];
    const JobDev& J = job_ref(jp, 0);
    const int n = *(volatile int32_t*)J.ovf_count;
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int id = J.ovf_list[i];
        if (id < 0) {
            const int64_t r = -(int64_t)id - 1;
            if (region_dense_cfg<KIND, DIM, CFG>(J, r, sm, threadIdx.x))
                alone_cfg<KIND, DIM, CFG>(J, r, w, fb[w], lane);
            __syncthreads();
        }
    }
    for (int i = blockIdx.x * NW + w; i < n; i += gridDim.x * NW) {
        const int id = J.ovf_list[i];
        if (id >= 0)
            alone_cfg<KIND, DIM, CFG>(J, id / NW, id % NW, fb[w], lane);
    }
}

template <int KIND, int DIM>
hipError_t launch_single_cfg(const JobDev& job, const JobDev* jd, hipStream_t s, bool fallback)
{
    const unsigned grid = fallback ? kFallbackGrid : (unsigned)job.nregions;
    if (fallback) {
        switch (job.cfg) {
        case 0: k_label_fallback<KIND, DIM, 0><<<grid, NT, 0, s>>>(jd); break;
        case 1: k_label_fallback<KIND, DIM, 1><<<grid, NT, 0, s>>>(jd); break;
        case 2: k_label_fallback<KIND, DIM, 2><<<grid, NT, 0, s>>>(jd); break;
        default: k_label_fallback<KIND, DIM, 3><<<grid, NT, 0, s>>>(jd); break;
        }
    } else {
        switch (job.cfg) {
        case 0: k_label_single<KIND, DIM, 0><<<grid, NT, 0, s>>>(jd); break;
        case 1: k_label_single<KIND, DIM, 1><<<grid, NT, 0, s>>>(jd); break;
        case 2: k_label_single<KIND, DIM, 2><<<grid, NT, 0, s>>>(jd); break;
        default: k_label_single<KIND, DIM, 3><<<grid, NT, 0, s>>>(jd); break;
        }
    }
    return hipGetLastError();
}

template <int DIM>
hipError_t launch_single_dim(const JobDev& job, const JobDev* jd, hipStream_t s, bool fallback)
{
    if (job.kind == KIND_VORONOI)
        return launch_single_cfg<KV, DIM>(job, jd, s, fallback);
    if (job.kind == KIND_LAGUERRE)
        return launch_single_cfg<KL, DIM>(job, jd, s, fallback);
    if (job.jm_div)
        return launch_single_cfg<KJD, DIM>(job, jd, s, fallback);
    return launch_single_cfg<KJM, DIM>(job, jd, s, fallback);
}

}  // namespace

hipError_t launch_label_single(const JobDev& job, const JobDev* job_dev, hipStream_t s)
{
    if (job.nregions <= 0 || job.nregions > 0x7fffffffLL || !job_dev)
        return hipErrorInvalidValue;
    return job.ndim == 3 ? launch_single_dim<3>(job, job_dev, s, false)
                         : launch_single_dim<2>(job, job_dev, s, false);
}

hipError_t launch_label_fallback(const JobDev& job, const JobDev* job_dev, hipStream_t s)
{
    if (!job_dev)
        return hipErrorInvalidValue;
    return job.ndim == 3 ? launch_single_dim<3>(job, job_dev, s, true) : launch_single_dim<2>(job, job_dev, s, true);
}

}  // namespace vt
