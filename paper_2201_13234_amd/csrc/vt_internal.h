// vt_internal.h -- types and launchers shared by the host code and the
// kernels of the device library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vtess.h"

namespace vt {

enum { KIND_VORONOI = 0, KIND_LAGUERRE = 1, KIND_JM = 2 };
enum { ST_OK = 0, ST_INPUT = 5 };

// Largest number of candidate sites one wave holds in LDS at a time.
constexpr int CAP = 128;
constexpr int WAVE = 64;

// Device-side description of one diagram.  Plain old data: copied to the
// device as a kernel argument (single job) or as a table (batches).
struct JobDev {
    int32_t ndim, kind, bc, cfg;   // cfg: tile configuration id
    int32_t jm_div;                // Johnson-Mehl: 1 = divide by v, 0 = multiply by exact 1/v
    int32_t nsites, nbins;
    int32_t gather_margin;         // bins beyond the region's own in its first gather box (Laguerre)
    int32_t n[3];                  // voxels per axis (n[2] = 1 in 2D)
    int32_t nb[3];                 // bins per axis (nb[2] = 1 in 2D)
    int32_t nr[3];                 // regions (groups of four tiles) per axis
    int32_t pad1;
    double L[3], h[3], H[3];       // lengths, voxel size, half lengths
    double bs[3], inv_bs[3];       // bin side and its reciprocal
    double growth, rgrowth;        // v and 1/v
    int64_t nvox, nregions;
    int64_t region_begin;          // first region of this job in a batch enumeration
    int64_t site_begin;            // first sorted site of this job in a batch (0 for a single job)
    int64_t bin_begin;             // first bin of this job in a batch (0 for a single job)
    const double* coords;          // [nsites][ndim], caller input
    const double* param;           // [nsites] or null
    int32_t* labels;               // caller output
    double* keys;                  // caller output (winning key per voxel) or null
    int32_t* status;               // one word, written by the kernels
    int32_t* bin_count;            // [nbins] sites per bin (live sites after pruning)
    int32_t* bin_start;            // [nbins + 1], indexes `sites`
    int32_t* site_bin;             // [nsites]
    int32_t* site_rank;            // [nsites]
    double4* sites;                // sorted sites {x, y, z, param}
    int32_t* sidx;                 // sorted -> input index (0-based)
    unsigned long long* pbound;    // [2]: ordered bits of max(param), max(-param)
    int32_t* ovf_list;             // tiles left to the fallback kernel (region * 4 + tile)
    int32_t* ovf_count;            // their number
};

// Tile configurations: a lane labels `rows` runs of `run` voxels along x
// (consecutive in y); lanes along x, y, z (one wavefront per tile); tiles per
// region along x, y, z (one workgroup of four wavefronts per region).  Denser
// site sets need smaller tiles so that a tile's candidate list stays short.
struct TileShape { int run, lx, ly, lz, rows, rx, ry, rz; };
constexpr int kNumCfg = 4;
// 3D: 0 = 8x16x8 tiles (two rows per lane) in 16x16x16 regions;
//     1 = 8x8x8 tiles in 16x16x8 regions;
//     2 = 8x4x4 tiles (two voxels per lane) in 8x8x8 regions;
//     3 = 4x4x4 tiles (one voxel per lane) in 8x8x4 regions.
constexpr TileShape kShape3[kNumCfg] = {{8, 1, 8, 8, 2, 2, 1, 2}, {8, 1, 8, 8, 1, 2, 2, 1},
                                        {2, 4, 4, 4, 1, 1, 2, 2}, {1, 4, 4, 4, 1, 2, 2, 1}};
// 2D: 0 = 32x32 tiles (two rows per lane) in 64x64 regions;
//     1 = 32x16 tiles in 64x32 regions;
//     2 = 16x8 tiles (two voxels per lane) in 32x16 regions;
//     3 = 8x8 tiles (one voxel per lane) in 16x16 regions.
constexpr TileShape kShape2[kNumCfg] = {{8, 4, 16, 1, 2, 2, 2, 1}, {8, 4, 16, 1, 1, 2, 2, 1},
                                        {2, 8, 8, 1, 1, 2, 2, 1}, {1, 8, 8, 1, 1, 2, 2, 1}};

inline TileShape shape_of(int ndim, int cfg) { return ndim == 3 ? kShape3[cfg] : kShape2[cfg]; }

// Square root with IEEE rounding, for q >= 2^-500 (finite): Goldschmidt's
// iteration for sqrt and 1/(2 sqrt) from the hardware reciprocal square root
// estimate (one coupled step on g ~ sqrt(q), h ~ 1/(2 sqrt(q))), then two
// Markstein corrections g += (q - g*g) * h with the residual formed exactly
// by a fused multiply-add (Markstein, IA-64 and Elementary Functions, 2000).
// This is the method of the compiler's correctly rounded binary64 sqrt on
// gfx950, without its rescaling of tiny inputs and its fix-up for zero and
// infinity (neither is reachable for finite q above 2^-500); the tests
// compare it bit for bit with host IEEE results on exact squares, their
// neighbours, rounding midpoints and random bit patterns.
__device__ inline double sqrt_refined(double q)
{
    const double y = __builtin_amdgcn_rsq(q);
    double g = q * y;
    double h = y * 0.5;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, q);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, q);
    return __builtin_fma(d, h, g);
}

// sqrt(q) for q >= 0, IEEE rounded, through sqrt_refined where it applies.
__device__ inline double key_sqrt(double q)
{
    return q >= 0x1p-500 ? sqrt_refined(q) : sqrt(q);
}

// A periodic site coordinate brought into the unit cell [0, L): the
// L-periodic distance (App. A, eq. L-distance_def) is unchanged when a point
// moves by whole periods.  fmod is exact; r + L for r < 0 is the one rounding,
// and a sum that rounds up to L is the origin of the next period.
__device__ inline double cell_coord(double c, double L)
{
    if (c >= 0.0 && c < L)
        return c + 0.0;  // fmod(c, L) == c: skip its loop (-0.0 -> +0.0 as below)
    double r = fmod(c, L);
    if (r < 0.0) {
        r = r + L;
        if (r >= L)
            r = 0.0;
    }
    return r + 0.0;  // -0.0 -> +0.0
}

// ---- launchers (defined in the .hip files) ----
// Binning over one job (jobs_dev == nullptr, `single` used) or over njobs jobs
// whose sites are enumerated by site_prefix_dev ([njobs + 1], device).
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_bin_count(const JobDev& single, const JobDev* jobs_dev, int njobs,
                            const int64_t* site_prefix_dev, int64_t total_sites, hipStream_t s);
// Exclusive scan out[0..n] of in[0..n) in one launch; flags: flags_cap zeroed
// words (scan_flags_needed(n)), cleared by the caller before every scan.
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, unsigned long long* flags,
                       int64_t flags_cap, hipStream_t s);
int64_t scan_flags_needed(int64_t n);
hipError_t launch_bin_scatter(const JobDev& single, const JobDev* jobs_dev, int njobs,
                              const int64_t* site_prefix_dev, int64_t total_sites, hipStream_t s);
// Johnson-Mehl jobs: drop from their bins the sites that provably never win
// (after binning; other kinds are left alone).  total_bins covers all jobs.
hipError_t launch_jm_prune(const JobDev& single, const JobDev* jobs_dev, int njobs,
                           const int64_t* site_prefix_dev, int64_t total_sites, int64_t total_bins, hipStream_t s);

// Labelling: a single job (all its tiles; job_dev: the same record in device
// memory, unchanged until the kernels have run) or one group of a batch: jobs
// of one kernel variant (label_variant), dimension and tile configuration,
// contiguous in the device table with region_begin counted from 0 over the
// group.  ovf_list: 4 entries per region; ovf_count: one zeroed int.
hipError_t launch_label_single(const JobDev& job, const JobDev* job_dev, hipStream_t s);
hipError_t launch_label_fallback(const JobDev& job, const JobDev* job_dev, hipStream_t s);
hipError_t launch_label_group(const JobDev* jobs_dev, int njobs, int variant, int ndim, int cfg,
                              int64_t total_regions, int32_t* ovf_list, int32_t* ovf_count, hipStream_t s);
int label_variant(const JobDev& J);  // 0 Voronoi, 1 Laguerre, 2/3 Johnson-Mehl (multiply / divide by v)

}  // namespace vt
