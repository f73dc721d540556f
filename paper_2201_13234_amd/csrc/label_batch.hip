// label_batch.hip -- labelling kernels over a batch of diagrams.
//
// The host sorts a batch into groups of one kind, dimension and tile
// configuration (contiguous in the device job table) and launches one kernel
// per group, each compiled for its group only, with one workgroup per region
// of all the group's jobs (enumerated job after job).  Tiles left over (too
// many candidates for LDS) go to the group's overflow list and a fallback
// kernel.
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

// One workgroup per region of the group, as the single-job kernel: the
// hardware spreads the regions of all the group's jobs over the chip, and
// consecutive regions go to one XCD (xcd_unit) so that they share its L2.
template <int KIND, int DIM, int CFG>
__global__ __launch_bounds__(NT) void k_label_batch(const JobDev* __restrict__ jobs, int njobs)
{
    __shared__ Smem sm;
    const int64_t g = xcd_unit(blockIdx.x, gridDim.x);
    const int j = job_of_region(jobs, njobs, g);
    const JobDev& J = job_ref(jobs, j);
    region_cfg<KIND, DIM, CFG>(J, g - J.region_begin, g, sm, threadIdx.x);
}

// The overflow list of a group, as k_label_fallback: regions queued whole
// (-(g + 1), group-wide region g) first, one workgroup each, then tiles
// (g * 4 + tile), one wavefront each.
template <int KIND, int DIM, int CFG>
__global__ __launch_bounds__(NT) void k_label_batch_fallback(const JobDev* __restrict__ jobs, int njobs,
                                                             const int32_t* list, const int32_t* count)
{
    __shared__ Smem sm;
    __shared__ FallbackLds fb[NW];
    const int n = *(volatile const int32_t*)count;
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int id = list[i];
        if (id < 0) {
            const int64_t g = -(int64_t)id - 1;
            const int j = job_of_region(jobs, njobs, g);
            const JobDev& J = job_ref(jobs, j);
            if (region_dense_cfg<KIND, DIM, CFG>(J, g - J.region_begin, sm, threadIdx.x))
                alone_cfg<KIND, DIM, CFG>(J, g - J.region_begin, w, fb[w], lane);
            __syncthreads();
        }
    }
    for (int i = blockIdx.x * NW + w; i < n; i += gridDim.x * NW) {
        const int id = list[i];
        if (id >= 0) {
            const int64_t g = id / NW;
            const int j = job_of_region(jobs, njobs, g);
            const JobDev& J = job_ref(jobs, j);
            alone_cfg<KIND, DIM, CFG>(J, g - J.region_begin, id % NW, fb[w], lane);
        }
    }
}

template <int KIND, int DIM, int CFG>
hipError_t launch_group_cfg(const JobDev* jobs, int njobs, int64_t total, int32_t* ovf_list, int32_t* ovf_count,
                            hipStream_t s)
{
    k_label_batch<KIND, DIM, CFG><<<(unsigned)total, NT, 0, s>>>(jobs, njobs);
    k_label_batch_fallback<KIND, DIM, CFG><<<kFallbackGrid, NT, 0, s>>>(jobs, njobs, ovf_list, ovf_count);
    return hipGetLastError();
}

template <int KIND, int DIM>
hipError_t launch_group_kind(int cfg, const JobDev* jobs, int njobs, int64_t total, int32_t* ovf_list,
                             int32_t* ovf_count, hipStream_t s)
{
    switch (cfg) {
    case 0: return launch_group_cfg<KIND, DIM, 0>(jobs, njobs, total, ovf_list, ovf_count, s);
    case 1: return launch_group_cfg<KIND, DIM, 1>(jobs, njobs, total, ovf_list, ovf_count, s);
    case 2: return launch_group_cfg<KIND, DIM, 2>(jobs, njobs, total, ovf_list, ovf_count, s);
    default: return launch_group_cfg<KIND, DIM, 3>(jobs, njobs, total, ovf_list, ovf_count, s);
    }
}

template <int DIM>
hipError_t launch_group_dim(int variant, int cfg, const JobDev* jobs, int njobs, int64_t total, int32_t* ovf_list,
                            int32_t* ovf_count, hipStream_t s)
{
    switch (variant) {
    case KV: return launch_group_kind<KV, DIM>(cfg, jobs, njobs, total, ovf_list, ovf_count, s);
    case KL: return launch_group_kind<KL, DIM>(cfg, jobs, njobs, total, ovf_list, ovf_count, s);
    case KJM: return launch_group_kind<KJM, DIM>(cfg, jobs, njobs, total, ovf_list, ovf_count, s);
    default: return launch_group_kind<KJD, DIM>(cfg, jobs, njobs, total, ovf_list, ovf_count, s);
    }
}

}  // namespace

int label_variant(const JobDev& J)
{
    return J.kind == KIND_VORONOI ? KV : J.kind == KIND_LAGUERRE ? KL : (J.jm_div ? KJD : KJM);
}

hipError_t launch_label_group(const JobDev* jobs_dev, int njobs, int variant, int ndim, int cfg,
                              int64_t total_regions, int32_t* ovf_list, int32_t* ovf_count, hipStream_t s)
{
    if (total_regions <= 0 || njobs <= 0)
        return hipSuccess;
    if (variant < KV || variant > KJD || cfg < 0 || cfg >= kNumCfg || (ndim != 2 && ndim != 3) ||
        total_regions > 0x7fffffffLL)
        return hipErrorInvalidValue;
    return ndim == 3 ? launch_group_dim<3>(variant, cfg, jobs_dev, njobs, total_regions, ovf_list, ovf_count, s)
                     : launch_group_dim<2>(variant, cfg, jobs_dev, njobs, total_regions, ovf_list, ovf_count, s);
}

}  // namespace vt
