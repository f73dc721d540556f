// bin_internal.h -- the plain path's binning launchers (not part of the
// public ABI): the count with the work that needs no launch of its own
// folded in, a one-workgroup scan for small bin grids, and the scatter that
// publishes the job's status word.
#pragma once

#include "vt_internal.h"

namespace vt {

// Extra work of the single-job count kernel.  Every pointer is nullable.
struct CountTail {
    int32_t* status_acc;   // invalid sites are ORed here (a zeroed word) instead of into job.status
    JobDev* job_dst;       // the job's record, stored here for the labelling kernels
    int32_t* clear;        // clear_words words set to zero (the scratch of the next call)
    int64_t clear_words;
};

// Largest bin grid scanned by one workgroup (launch_scan_small): 16
// wavefronts of 16 rows of 256 counts (8 rows up to 32,768 bins).  Its counts
// are padded with zeros to count_words(nbins) words, whole wavefronts, and it
// writes count_words(nbins) + 1 words of the output.
constexpr int64_t kSmallScanMax = 65536;
inline int64_t small_scan_wave_counts(int64_t nbins) { return nbins <= 32768 ? 8 * 256 : 16 * 256; }
inline int64_t count_words(int64_t nbins)
{
    if (nbins > kSmallScanMax)
        return nbins;
    const int64_t w = small_scan_wave_counts(nbins);
    return (nbins + w - 1) / w * w;
}

// Counting pass over one job's sites (`job` as bound for this call), with
// the extra work of `tail`.
hipError_t launch_bin_count_single(const JobDev& job, const CountTail& tail, hipStream_t s);
// Exclusive scan out[0..n] of cnt[0..n) by one workgroup (n <= kSmallScanMax,
// cnt and out 16-byte aligned and sized as above).
hipError_t launch_scan_small(const int32_t* cnt, int32_t* out, int64_t n, hipStream_t s);
// Scatter of one job's sites; with status_acc given, also stores *status_acc
// into *job.status.
hipError_t launch_bin_scatter_single(const JobDev& job, const int32_t* status_acc, hipStream_t s);

}  // namespace vt
