// nd_internal.h -- the general path (any dimension, general period vectors):
// device-side job description and launchers (not part of the public ABI).
#pragma once

#include "vt_internal.h"

namespace vt {

// ---- any dimension (1 .. kMaxDim): the general path ----
constexpr int kMaxDim = 6;

// Device-side description of one diagram of the general path.
struct NdDev {
    int32_t ndim, kind, bc, jm_div;
    int32_t nsites, nbins;
    int32_t T[kMaxDim];            // tile voxels per axis (powers of two; product / vpt <= 256 threads)
    int32_t nb[kMaxDim];           // bins per axis
    int64_t n[kMaxDim];            // voxels per axis
    int64_t nt[kMaxDim];           // tiles per axis
    int64_t ntiles;
    double L[kMaxDim], h[kMaxDim], H[kMaxDim];
    double bs[kMaxDim], inv_bs[kMaxDim];
    double growth, rgrowth;
    // General period vectors (lattice != 0; App. A, eq. L-distance_def).  The
    // bins, L, H, bs and inv_bs above then live in fractional coordinates
    // (period 1 per axis).
    int32_t lattice;
    int32_t vpt;                   // voxels per thread (1 or 2), the second T[0] / vpt further along axis 0
    double P[kMaxDim][kMaxDim];    // P[i][a]: component a of period vector i
    double hv[kMaxDim][kMaxDim];   // P[i][a] / n_i: voxel steps
    double Pinv[kMaxDim][kMaxDim]; // Pinv[i][a]: fractional coordinate i per Cartesian a
    double rown[kMaxDim];          // norm of row i of Pinv
    double cell_d;                 // sum of |P_i|
    const double* coords;          // [nsites][ndim], caller input
    const double* param;           // [nsites] or null
    int32_t* labels;               // caller output
    double* keys;                  // caller output or null
    int32_t* status;               // one word, written by the kernels
    int32_t* bin_count;            // [nbins]
    int32_t* bin_start;            // [nbins + 1]
    int32_t* site_bin;             // [nsites]
    int32_t* site_rank;            // [nsites]
    double* sc;                    // [nsites][ndim] sorted coordinates (inside the cell unless lattice)
    double* sf;                    // [nsites][ndim] sorted fractional coordinates (lattice only)
    double* sp;                    // [nsites] sorted parameters
    int32_t* sidx;                 // sorted -> input index
    unsigned long long* pbound;    // [3]: ordered bits of max(param), max(-param), max |coordinate|
};

// Binning of the general path: status_acc is a zeroed word that collects
// invalid sites and that the scatter stores into *J.status; the count also
// clears clear_words words at `clear` (16-byte aligned; nullable).
hipError_t launch_nd_bin_count(const NdDev& J, int32_t* status_acc, int32_t* clear, int64_t clear_words,
                               hipStream_t s);
hipError_t launch_nd_bin_scatter(const NdDev& J, const int32_t* status_acc, hipStream_t s);
hipError_t launch_nd_label(const NdDev& J, hipStream_t s);

}  // namespace vt
