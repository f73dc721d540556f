// label_batch.hip -- persistent labelling kernels over a batch of diagrams.
//
// The host sorts a batch into groups of one kind, dimension and tile
// configuration (contiguous in the device job table) and launches one
// persistent kernel per group, each compiled for its group only.  A group's
// regions are enumerated job after job and cut into eight ranges, one per XCD;
// each workgroup takes regions of its own XCD's range from an atomic counter,
// then helps the other ranges.  Tiles left over (too many candidates for LDS)
// go to the group's overflow list and a fallback kernel.
#include "label_core.h"

namespace vt {

namespace {

__device__ inline int job_of_region(const JobDev* jobs, int njobs, int64_t g)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].region_begin <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// The job's record is held in scalar registers across the region loop, and
// without a bound the scalar registers that spill into vector registers halve
// the occupancy; asking for 4 waves per SIMD (3 for Laguerre, measured)
// trades that for a few vector-register spills and is faster.
template <int KIND, int DIM, int CFG>
__global__ __launch_bounds__(NT, KIND == KL ? 3 : 4) void k_label_batch(const JobDev* __restrict__ jobs, int njobs, int64_t total,
                                                    int32_t* counters)
{
    __shared__ Smem sm;
    __shared__ int64_t got;
    const int tid = threadIdx.x;
    const int home = blockIdx.x & 7;
    for (int probe = 0; probe < 8; ++probe) {
        const int x = (home + probe) & 7;
        const int64_t rb = total * x / 8, re = total * (x + 1) / 8;
        for (;;) {
            if (tid == 0)
                got = rb + (int64_t)atomicAdd(&counters[x], 1);
            __syncthreads();
            // the same for every lane: say so, so that the region's geometry
            // and its job's record stay in scalar registers
            const int64_t gv = got;
            const int64_t g = ((int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(gv >> 32)) << 32) |
                              (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)gv);
            __syncthreads();
            if (g >= re)
                break;
            const int j = job_of_region(jobs, njobs, g);
            const JobDev J = jobs[j];  // by value: read once, not through a generic pointer
            region_cfg<KIND, DIM, CFG>(J, g - J.region_begin, g, sm, tid);
            __syncthreads();
        }
    }
}

// Fallback over a group's overflow list (entries are group-wide region * 4 + tile).
template <int KIND, int DIM, int CFG>
__global__ __launch_bounds__(WAVE) void k_label_batch_fallback(const JobDev* __restrict__ jobs, int njobs,
                                                               const int32_t* list, const int32_t* count)
{
    __shared__ FallbackLds S;
    const int n = *(volatile const int32_t*)count;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int id = list[i];
        const int64_t g = id / NW;
        const int j = job_of_region(jobs, njobs, g);
        const JobDev J = jobs[j];
        alone_cfg<KIND, DIM, CFG>(J, g - J.region_begin, id % NW, S, threadIdx.x);
        __syncthreads();
    }
}

template <int KIND, int DIM, int CFG>
hipError_t launch_group_cfg(const JobDev* jobs, int njobs, int64_t total, int32_t* counters, int32_t* ovf_list,
                            int32_t* ovf_count, int grid, hipStream_t s)
{
    k_label_batch<KIND, DIM, CFG><<<grid, NT, 0, s>>>(jobs, njobs, total, counters);
    k_label_batch_fallback<KIND, DIM, CFG><<<kFallbackGrid, WAVE, 0, s>>>(jobs, njobs, ovf_list, ovf_count);
    return hipGetLastError();
}

template <int KIND, int DIM>
hipError_t launch_group_kind(int cfg, const JobDev* jobs, int njobs, int64_t total, int32_t* counters,
                             int32_t* ovf_list, int32_t* ovf_count, int grid, hipStream_t s)
{
    switch (cfg) {
    case 0: return launch_group_cfg<KIND, DIM, 0>(jobs, njobs, total, counters, ovf_list, ovf_count, grid, s);
    case 1: return launch_group_cfg<KIND, DIM, 1>(jobs, njobs, total, counters, ovf_list, ovf_count, grid, s);
    case 2: return launch_group_cfg<KIND, DIM, 2>(jobs, njobs, total, counters, ovf_list, ovf_count, grid, s);
    default: return launch_group_cfg<KIND, DIM, 3>(jobs, njobs, total, counters, ovf_list, ovf_count, grid, s);
    }
}

template <int DIM>
hipError_t launch_group_dim(int variant, int cfg, const JobDev* jobs, int njobs, int64_t total, int32_t* counters,
                            int32_t* ovf_list, int32_t* ovf_count, int grid, hipStream_t s)
{
    switch (variant) {
    case KV: return launch_group_kind<KV, DIM>(cfg, jobs, njobs, total, counters, ovf_list, ovf_count, grid, s);
    case KL: return launch_group_kind<KL, DIM>(cfg, jobs, njobs, total, counters, ovf_list, ovf_count, grid, s);
    case KJM: return launch_group_kind<KJM, DIM>(cfg, jobs, njobs, total, counters, ovf_list, ovf_count, grid, s);
    default: return launch_group_kind<KJD, DIM>(cfg, jobs, njobs, total, counters, ovf_list, ovf_count, grid, s);
    }
}

}  // namespace

int label_variant(const JobDev& J)
{
    return J.kind == KIND_VORONOI ? KV : J.kind == KIND_LAGUERRE ? KL : (J.jm_div ? KJD : KJM);
}

int label_batch_grid(int device)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    return cus * 4;
}

hipError_t launch_label_group(const JobDev* jobs_dev, int njobs, int variant, int ndim, int cfg,
                              int64_t total_regions, int32_t* counters, int32_t* ovf_list, int32_t* ovf_count,
                              int grid, hipStream_t s)
{
    if (total_regions <= 0 || njobs <= 0)
        return hipSuccess;
    if (variant < KV || variant > KJD || cfg < 0 || cfg >= kNumCfg || (ndim != 2 && ndim != 3))
        return hipErrorInvalidValue;
    if (total_regions < grid)
        grid = (int)total_regions;
    return ndim == 3 ? launch_group_dim<3>(variant, cfg, jobs_dev, njobs, total_regions, counters, ovf_list,
                                           ovf_count, grid, s)
                     : launch_group_dim<2>(variant, cfg, jobs_dev, njobs, total_regions, counters, ovf_list,
                                           ovf_count, grid, s);
}

}  // namespace vt
