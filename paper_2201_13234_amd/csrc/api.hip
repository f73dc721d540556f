// api.hip -- host side of the C ABI declared in include/vtess.h: argument
// checks, planning (bin grid, tile grid), scratch ownership, launch
// sequencing, the resident-bins objects used by the serving loop, and the
// autotuner with its JSON cache.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bin_internal.h"
#include "nd_internal.h"
#include "vtess.h"

using vt::JobDev;

namespace {

thread_local std::string g_last_error;

vt_status fail(vt_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

vt_status hip_fail(hipError_t e, const char* what)
{
    return fail(VT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define VT_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess)                          \
            return hip_fail(e_, #call);                \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Scratch of vt_tessellate_noalloc: a file-scope device array, one copy per
// device, allocated by the runtime when this code object is loaded on that
// device and held until the process ends.  Host code never uses the name
// itself as an address (on the host it is only a stand-in): vt_create asks the
// runtime for its address on the device once (hipGetSymbolAddress, with that
// device current) and the entry point passes that address to the kernels.
constexpr size_t kNoallocBytes = VT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices];  // device address of `scratch` per device (null until set up)

// Carves sub-arrays out of one allocation.
struct Carver {
    size_t off = 0;
    template <class T>
    size_t take(int64_t count, size_t align = 256)
    {
        off = align_up(off, align);
        size_t at = off;
        off += (size_t)std::max<int64_t>(count, 0) * sizeof(T);
        return at;
    }
};

struct TuneEntry {
    int ndim, kind, bc, size_cls, dens_cls;
    int cfg;
    double bin_factor;
    int gather_margin;  // Laguerre first gather box margin in bins (0: the default rule)
    double ms;          // tuned round time
    double default_ms;  // the built-in plan's round time on the same samples
};

int size_class(int64_t nvox) { return (int)std::floor(std::log2((double)std::max<int64_t>(nvox, 1)) / 2.0); }
int dens_class(int64_t nvox, int64_t ns)
{
    return (int)std::floor(std::log2((double)std::max<int64_t>(nvox, 1) / (double)std::max<int64_t>(ns, 1)));
}

}  // namespace

struct vt_ctx {
    int device = 0;
    // scratch of the plain path and of batch binning
    void* arena = nullptr;
    size_t arena_cap = 0;
    // pinned staging for job tables; the event marks the last copy out of it
    void* pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t staging_evt = nullptr;
    bool staging_used = false;
    int force_cfg = -1;
    double force_bin = 0.0;
    int force_margin = 0;      // Laguerre gather margin forced by the autotuner (0: none)
    bool skip_tune = false;    // plan without the tuning table (the autotuner's default rounds)
    std::vector<TuneEntry> tune;
    // The plain and general paths keep two slots of zeroed scratch (bin
    // counts, bounds, counters) at the start of the arena, laid out for the
    // path that used them last (slot_owner): a call uses one and its count
    // kernel clears the other for the next call.  slot_clean[k]: bytes of
    // slot k known to be zero (0 after any other use of the arena).  Calls
    // captured into a graph use a third slot, which they clear themselves.
    size_t slot_cap = 0;
    size_t slot_clean[2] = {0, 0};
    int slot_next = 0;
    int slot_owner = -1;  // path whose layout the slots follow: 0 plain, 1 general, -1 none
    // this device's copy of the static scratch (vt_tessellate_noalloc)
    void* noalloc = nullptr;
    // phase timing: three events per recorded call
    bool profile = false;
    std::vector<hipEvent_t> prof_events;
    size_t prof_used = 0;
};

struct vt_bins {
    JobDev job;
    void* mem = nullptr;
};

namespace {

bool is_pow2_scale(double v)
{
    int e = 0;
    double m = std::frexp(v, &e);
    return m == 0.5 && e >= -60 && e <= 60;
}

const TuneEntry* find_tune(const vt_ctx* ctx, const vt_job* j, int64_t nvox)
{
    const int sc = size_class(nvox), dc = dens_class(nvox, j->nsites);
    for (const TuneEntry& t : ctx->tune)
        if (t.ndim == j->ndim && t.kind == j->kind && t.bc == (j->bc ? 1 : 0) && t.size_cls == sc &&
            t.dens_cls == dc)
            return &t;
    return nullptr;
}

// Tile configuration and bin size: forced, tuned, or default.  The default
// tile shrinks as sites get denser (voxels per site, divided by 1.5 for
// Laguerre and Johnson-Mehl diagrams, whose weights and times let farther
// sites compete), so that a tile's candidate list stays within its capacity
// or overflows to the fallback rarely enough to pay.  The 3D thresholds and
// bin factors are the fastest measured per kind on uniform random sites
// (384^3 and 512^3 grids): larger bins than the mean spacing mean fewer bin
// visits per region, until dense grids overflow tiles; a Johnson-Mehl
// diagram, whose cells reach further, labels best with 8x8x8 tiles.
// Batched launches group jobs by configuration, so the same choice holds
// there.
void choose_params(const vt_ctx* ctx, const vt_job* j, int64_t nvox, int* cfg_out, double* bf_out,
                   int* margin_out = nullptr)
{
    const double vps = (double)nvox / (double)std::max<int64_t>(j->nsites, 1) /
                       (j->kind == VT_VORONOI ? 1.0 : 1.5);
    int cfg;
    double bf = 1.0;
    if (j->ndim == 3) {
        if (j->kind == VT_VORONOI) {
            cfg = vps >= 1100.0 ? 0 : (vps >= 145.0 ? 1 : (vps >= 50.0 ? 2 : 3));
            // 1.6 spacings below 2,500 voxels per site (M2 at 1,342: 0.718 ->
            // 0.692 ms against 1.4), 1.4 in sparser grids, 1.2 in the dense
            // end of 8x8x8 tiles, where larger bins overflow tiles
            bf = vps >= 2500.0 ? 1.4 : (vps >= 225.0 ? 1.6 : 1.2);
        } else if (j->kind == VT_LAGUERRE) {
            // (the region gather leaves out sites that provably lose when a
            // round would overflow, which keeps these larger tiles usable
            // where a few heavy weights set the reach for everyone)
            cfg = vps >= 800.0 ? 0 : (vps >= 200.0 ? 1 : (vps >= 33.0 ? 2 : 3));
            // large bins only where sites are sparse: denser jobs would gather
            // many more sites than their tiles need
            bf = vps >= 2000.0 ? 2.0 : 1.2;
        } else {
            cfg = vps >= 130.0 ? 1 : (vps >= 45.0 ? 2 : 3);
            bf = 1.0;
        }
    } else {
        // measured per kind on 512^2 to 4096^2 grids from 12 to 300 voxels
        // per site (same-box comparisons against the former common
        // thresholds 144 / 81 / 20)
        if (j->kind == VT_VORONOI)
            cfg = vps >= 144.0 ? 0 : (vps >= 60.0 ? 1 : (vps >= 20.0 ? 2 : 3));
        else if (j->kind == VT_LAGUERRE)
            cfg = vps >= 90.0 ? 0 : (vps >= 38.0 ? 1 : (vps >= 20.0 ? 2 : 3));
        else
            cfg = vps >= 200.0 ? 0 : (vps >= 45.0 ? 1 : (vps >= 9.5 ? 2 : 3));
        // measured on 2048^2 to 8192^2 grids with 2,000 to 100,000 sites:
        // Voronoi and Laguerre label fastest from bins of 1.6 spacings (up
        // to 12 % faster than one spacing), Johnson-Mehl from 1.2 to 1.4
        bf = j->kind == VT_JOHNSON_MEHL ? 1.2 : 1.6;
    }
    if (cfg >= 2)  // small regions: bins near one spacing keep the region list short
        bf = j->ndim == 3 ? 1.2 : 1.0;  // 3D measured 2-4 % faster at 1.2, 2D level
    int margin = 0;
    if (ctx) {  // planning without a context takes the defaults
        const TuneEntry* t = ctx->skip_tune ? nullptr : find_tune(ctx, j, nvox);
        if (t) {
            cfg = t->cfg;
            bf = t->bin_factor;
            margin = t->gather_margin;
        }
        if (ctx->force_cfg >= 0)
            cfg = ctx->force_cfg;
        if (ctx->force_bin > 0.0)
            bf = ctx->force_bin;
        if (ctx->force_margin > 0)
            margin = ctx->force_margin;
    }
    if (cfg < 0 || cfg >= vt::kNumCfg)
        cfg = 0;
    // Laguerre's first gather box: two rings of bins near the mean spacing,
    // one with larger bins (whose two rings would overflow the region list)
    if (margin < 1 || margin > 2)
        margin = bf <= 1.25 ? 2 : 1;
    *cfg_out = cfg;
    *bf_out = bf;
    if (margin_out)
        *margin_out = margin;
}

// A scalar inside the supported scale [VT_SCALE_MIN, VT_SCALE_MAX] (see the
// header): squared distances, keys and rounding margins then stay finite
// normal numbers.
bool in_scale(double x)
{
    return x >= VT_SCALE_MIN && x <= VT_SCALE_MAX;
}

// Checks the scalars of a job and fills the geometry of its device record.
vt_status plan_job(const vt_ctx* ctx, const vt_job* j, JobDev* d)
{
    if (!j)
        return fail(VT_ERR_INVALID, "job is NULL");
    if (j->ndim != 2 && j->ndim != 3)
        return fail(VT_ERR_INVALID, "ndim must be 2 or 3");
    if (j->kind < VT_VORONOI || j->kind > VT_JOHNSON_MEHL)
        return fail(VT_ERR_INVALID, "unknown diagram kind");
    if (j->bc != VT_NONPERIODIC && j->bc != VT_PERIODIC)
        return fail(VT_ERR_INVALID, "unknown boundary mode");
    if (j->nsites < 1 || j->nsites > 0x7fffffffLL)
        return fail(VT_ERR_INVALID, "nsites must be in [1, 2^31-1]");
    if (!j->coords || !j->labels)
        return fail(VT_ERR_INVALID, "coords and labels must be device pointers");
    if (j->kind != VT_VORONOI && !j->param)
        return fail(VT_ERR_INVALID, "param is required for Laguerre and Johnson-Mehl");
    if (j->kind == VT_JOHNSON_MEHL && !in_scale(j->growth))
        return fail(VT_ERR_INVALID, "growth rate must lie in [2^-200, 2^200]");
    std::memset(d, 0, sizeof *d);
    d->ndim = j->ndim;
    d->kind = j->kind;
    d->bc = j->bc ? 1 : 0;
    int64_t nvox = 1;
    double V = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (a < j->ndim) {
            if (j->n[a] < 1 || j->n[a] > (1 << 30))
                return fail(VT_ERR_INVALID, "n[a] must be in [1, 2^30]");
            if (!in_scale(j->L[a]))
                return fail(VT_ERR_INVALID, "L[a] must lie in [2^-200, 2^200]");
            d->n[a] = (int32_t)j->n[a];
            d->L[a] = j->L[a];
            d->h[a] = j->L[a] / (double)j->n[a];
            d->H[a] = 0.5 * j->L[a];
        } else {
            d->n[a] = 1;
            d->L[a] = 1.0;
            d->h[a] = 1.0;
            d->H[a] = 0.5;
        }
        // checked before the product: three axes of up to 2^30 overflow int64
        if (nvox > ((int64_t)1 << 40) / d->n[a])
            return fail(VT_ERR_INVALID, "more than 2^40 voxels");
        nvox *= d->n[a];
        V *= d->L[a];
    }
    d->nvox = nvox;
    d->nsites = (int32_t)j->nsites;
    d->growth = j->kind == VT_JOHNSON_MEHL ? j->growth : 1.0;
    d->rgrowth = 1.0 / d->growth;
    d->jm_div = (j->kind == VT_JOHNSON_MEHL && !is_pow2_scale(d->growth)) ? 1 : 0;

    int cfg, margin;
    double bf;
    choose_params(ctx, j, nvox, &cfg, &bf, &margin);
    d->cfg = cfg;
    // Laguerre regions start their gather two bins out when the bins are near
    // the mean spacing (3-16 % faster on 384^3 grids from 167 to 1,067
    // voxels per site divided by 1.5), one bin out with larger bins, whose
    // first box would overflow the region list (or as tuned)
    d->gather_margin = j->kind == VT_LAGUERRE ? margin : 1;

    // Bins: side ~ bf times the mean site spacing (V / N)^(1/d), at most
    // 2^20 per axis and about 4 N + 64 in total.
    const double spacing = std::pow(V / (double)j->nsites, 1.0 / j->ndim) * bf;
    int64_t nbins = 1;
    for (int a = 0; a < 3; ++a) {
        int nb = 1;
        if (a < j->ndim) {
            double f = std::floor(j->L[a] / spacing + 0.5);
            nb = (int)std::min(std::max(f, 1.0), (double)(1 << 20));
        }
        d->nb[a] = nb;
        nbins *= nb;
    }
    while (nbins > 4 * (int64_t)j->nsites + 64) {
        nbins = 1;
        for (int a = 0; a < j->ndim; ++a) {
            d->nb[a] = std::max(1, d->nb[a] * 3 / 4);
            nbins *= d->nb[a];
        }
    }
    for (int a = 0; a < 3; ++a) {
        d->bs[a] = d->L[a] / (double)d->nb[a];
        d->inv_bs[a] = (double)d->nb[a] / d->L[a];
    }
    d->nbins = (int32_t)nbins;

    const vt::TileShape sh = vt::shape_of(j->ndim, cfg);
    const int R[3] = {sh.run * sh.lx * sh.rx, sh.ly * sh.rows * sh.ry, j->ndim == 3 ? sh.lz * sh.rz : 1};
    int64_t nregions = 1;
    for (int a = 0; a < 3; ++a) {
        d->nr[a] = (d->n[a] + R[a] - 1) / R[a];
        nregions *= d->nr[a];
    }
    d->nregions = nregions;
    d->coords = j->coords;
    d->param = j->param;
    d->labels = j->labels;
    d->keys = j->keys;
    return VT_OK;
}

vt_status ensure_scratch(vt_ctx* ctx, size_t bytes)
{
    if (bytes <= ctx->arena_cap)
        return VT_OK;
    // Growing replaces memory that queued work may still use.
    VT_HIP(hipDeviceSynchronize());
    ctx->slot_clean[0] = ctx->slot_clean[1] = 0;
    if (ctx->arena)
        VT_HIP(hipFree(ctx->arena));
    ctx->arena = nullptr;
    ctx->arena_cap = 0;
    size_t cap = align_up(bytes + bytes / 4, 1 << 20);
    if (hipMalloc(&ctx->arena, cap) != hipSuccess) {
        ctx->arena = nullptr;
        return fail(VT_ERR_NOMEM, "scratch allocation failed");
    }
    ctx->arena_cap = cap;
    return VT_OK;
}

vt_status ensure_pinned(vt_ctx* ctx, size_t bytes)
{
    if (ctx->staging_used)
        VT_HIP(hipEventSynchronize(ctx->staging_evt));
    ctx->staging_used = false;
    if (bytes <= ctx->pinned_cap)
        return VT_OK;
    if (ctx->pinned)
        VT_HIP(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_cap = 0;
    size_t cap = align_up(bytes + bytes / 4, 1 << 16);
    if (hipHostMalloc(&ctx->pinned, cap, hipHostMallocDefault) != hipSuccess) {
        ctx->pinned = nullptr;
        return fail(VT_ERR_NOMEM, "pinned staging allocation failed");
    }
    ctx->pinned_cap = cap;
    return VT_OK;
}

// The words of one job that must start at zero: parameter bounds, the
// count's status accumulator, the overflow count, the bin counts (padded
// with zeros for the one-workgroup scan) and the flags of the multi-workgroup
// scan.
struct SlotLayout {
    size_t pbound, sacc, ovf_count, bin_count, partial, bytes;
    int64_t partial_cap;
};

SlotLayout slot_layout(const JobDev& d)
{
    SlotLayout Z;
    Carver c;
    Z.pbound = c.take<unsigned long long>(2);
    Z.sacc = c.take<int32_t>(1, 4);
    Z.ovf_count = c.take<int32_t>(1, 4);
    Z.bin_count = c.take<int32_t>(vt::count_words(d.nbins));
    Z.partial_cap = vt::scan_flags_needed((int64_t)d.nbins);
    Z.partial = c.take<unsigned long long>(Z.partial_cap, 8);
    Z.bytes = align_up(c.off, 256);
    return Z;
}

// Binning arrays of one job carved from `base` (device memory): the job's
// record, one or three slots of slot_bytes each for the words that start at
// zero (slot_layout), then the rest.
struct SingleLayout {
    SlotLayout z;
    size_t job, slot[3], status, bin_start, site_bin, site_rank, sites, sidx, ovf_list, total;
};

SingleLayout single_layout(const JobDev& d, size_t slot_bytes, int nslots)
{
    SingleLayout L;
    Carver c;
    L.z = slot_layout(d);
    // written by the count kernel, read by the labelling kernels
    L.job = c.take<JobDev>(1);
    for (int k = 0; k < 3; ++k)
        L.slot[k] = k == 0 || nslots == 3 ? c.take<char>((int64_t)slot_bytes) : L.slot[0];
    // the job's status when the caller gives no word of its own
    L.status = c.take<int32_t>(1, 4);
    // (the one-workgroup scan writes whole rows: count_words(nbins) + 1 words)
    L.bin_start = c.take<int32_t>(vt::count_words(d.nbins) + 1);
    L.site_bin = c.take<int32_t>(d.nsites);
    L.site_rank = c.take<int32_t>(d.nsites);
    L.sites = c.take<double4>(d.nsites);
    L.sidx = c.take<int32_t>(d.nsites);
    L.ovf_list = c.take<int32_t>(d.nregions * 4);
    L.total = align_up(c.off, 256);
    return L;
}

void bind_single(JobDev& d, char* base, const SingleLayout& L, int slot, int32_t* status_dev)
{
    char* z = base + L.slot[slot];
    d.pbound = (unsigned long long*)(z + L.z.pbound);
    d.status = status_dev ? status_dev : (int32_t*)(base + L.status);
    d.bin_count = (int32_t*)(z + L.z.bin_count);
    d.bin_start = (int32_t*)(base + L.bin_start);
    d.site_bin = (int32_t*)(base + L.site_bin);
    d.site_rank = (int32_t*)(base + L.site_rank);
    d.sites = (double4*)(base + L.sites);
    d.sidx = (int32_t*)(base + L.sidx);
    d.ovf_count = (int32_t*)(z + L.z.ovf_count);
    d.ovf_list = (int32_t*)(base + L.ovf_list);
}

// Clears nwords words from zero_begin and the word *extra (if given).
__global__ void k_prepare(int32_t* zero_begin, int64_t nwords, int32_t* extra)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < nwords; k += stride)
        zero_begin[k] = 0;
    if (i == 0 && extra)
        *extra = 0;
}

hipError_t launch_prepare(int32_t* zero_begin, int64_t nwords, int32_t* extra, hipStream_t s)
{
    int64_t g = (nwords + 255) / 256;
    g = std::min<int64_t>(std::max<int64_t>(g, 1), 4096);
    k_prepare<<<(unsigned)g, 256, 0, s>>>(zero_begin, nwords, extra);
    return hipGetLastError();
}

// ---- the zeroed slots of the plain and general paths ----
//
// Each path lays out three slots of ctx->slot_cap bytes for the words that
// must start at zero: a call uses slot 0 or 1 and its count kernel clears
// the other for the next call; a call captured into a graph uses slot 2 and
// clears it itself, since its replays may come in any order with other calls.

// Settles the slots' layout for a call of path `owner` whose zeroed words
// take zbytes: another path's layout or a larger slot makes every slot
// unknown.
void slots_for(vt_ctx* ctx, int owner, size_t zbytes)
{
    if (ctx->slot_owner != owner || zbytes > ctx->slot_cap) {
        ctx->slot_owner = owner;
        ctx->slot_cap = std::max(ctx->slot_cap, zbytes);
        ctx->slot_clean[0] = ctx->slot_clean[1] = 0;
    }
}

struct SlotUse {
    int slot;
    bool zeroed, capturing;
};

// The slot of this call (after the arena is in place), whether it is known
// to be zero, and whether the stream is capturing (a stream whose capture
// state cannot be read is taken as capturing).  Nothing is known to be zero
// until slot_end: a failed launch in between leaves the slots unknown.
SlotUse slot_begin(vt_ctx* ctx, size_t zbytes, hipStream_t s)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    bool capturing = true;
    if (hipStreamIsCapturing(s, &cap) == hipSuccess)
        capturing = cap != hipStreamCaptureStatusNone;
    else
        (void)hipGetLastError();
    SlotUse u;
    u.capturing = capturing;
    u.slot = capturing ? 2 : ctx->slot_next;
    u.zeroed = !capturing && ctx->slot_clean[u.slot] >= zbytes;
    ctx->slot_clean[0] = ctx->slot_clean[1] = 0;
    return u;
}

// Every launch of the call is queued: the other slot is zero for the next.
void slot_end(vt_ctx* ctx, const SlotUse& u, size_t zbytes)
{
    if (u.capturing)
        return;
    ctx->slot_clean[u.slot ^ 1] = zbytes;
    ctx->slot_next = u.slot ^ 1;
}

// Count, scan and scatter the sites of one job (its arrays bound to `slot`).
// Unless `zeroed`, the slot is cleared first; with clear_other, the count
// kernel clears the other slot (its first L.z.bytes) for the next call.
// The count also stores the job's record and accumulates the input status in
// the slot; the scatter publishes that status in *d.status.  Small bin grids
// are scanned by one workgroup, larger ones by the multi-workgroup scan.
vt_status bin_single(const JobDev& d, char* base, const SingleLayout& L, int slot, bool zeroed, bool clear_other,
                     hipStream_t s)
{
    char* z = base + L.slot[slot];
    if (!zeroed)
        VT_HIP(launch_prepare((int32_t*)z, (int64_t)(L.z.bytes / 4), nullptr, s));
    vt::CountTail t;
    t.status_acc = (int32_t*)(z + L.z.sacc);
    t.job_dst = (JobDev*)(base + L.job);
    t.clear = clear_other ? (int32_t*)(base + L.slot[slot ^ 1]) : nullptr;
    t.clear_words = clear_other ? (int64_t)(L.z.bytes / 4) : 0;
    VT_HIP(vt::launch_bin_count_single(d, t, s));
    if (d.nbins <= vt::kSmallScanMax)
        VT_HIP(vt::launch_scan_small(d.bin_count, d.bin_start, d.nbins, s));
    else
        VT_HIP(vt::launch_scan(d.bin_count, d.bin_start, d.nbins, (unsigned long long*)(z + L.z.partial),
                               L.z.partial_cap, s));
    VT_HIP(vt::launch_bin_scatter_single(d, t.status_acc, s));
    if (d.kind == vt::KIND_JM)
        VT_HIP(vt::launch_jm_prune(d, nullptr, 1, nullptr, d.nsites, d.nbins, s));
    return VT_OK;
}

__global__ void k_probe(const double* x, const double* den, double* so, double* dq, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        so[i] = vt::key_sqrt(x[i]);  // the square root the Johnson-Mehl keys use
        dq[i] = x[i] / den[i];
    }
}

// out[order[k]] = status of table entry k.
__global__ void k_copy_status(const JobDev* jobs, int n, const int32_t* order, int32_t* out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n)
        out[order[k]] = *jobs[k].status;
}

// Stream-ordered device allocation for per-call tables (freed by the caller
// with hipFreeAsync after the launches that read it).
vt_status alloc_table(size_t bytes, hipStream_t s, void** dev)
{
    *dev = nullptr;
    if (hipMallocAsync(dev, bytes, s) != hipSuccess) {
        *dev = nullptr;
        return fail(VT_ERR_NOMEM, "table allocation failed");
    }
    return VT_OK;
}

// Copies `bytes` of host data to the device through the pinned staging buffer.
vt_status stage_copy(vt_ctx* ctx, void* dev, const void* host, size_t bytes, hipStream_t s)
{
    vt_status st = ensure_pinned(ctx, bytes);
    if (st != VT_OK)
        return st;
    std::memcpy(ctx->pinned, host, bytes);
    VT_HIP(hipMemcpyAsync(dev, ctx->pinned, bytes, hipMemcpyHostToDevice, s));
    VT_HIP(hipEventRecord(ctx->staging_evt, s));
    ctx->staging_used = true;
    return VT_OK;
}

// One launch group of a batch: jobs of one kernel variant, dimension and tile
// configuration, contiguous in the table.
struct Group {
    int first, count, variant, ndim, cfg;
    int64_t regions, ovf_off;
};

// Orders a batch's jobs into launch groups (stable within a group), numbers
// each group's regions from 0 (region_begin) and places its overflow list.
// order[k] is the caller's index of table entry k; group_of[k] its group.
void make_groups(std::vector<JobDev>& tab, std::vector<int>& order, std::vector<int>& group_of,
                 std::vector<Group>& groups)
{
    const int n = (int)tab.size();
    auto key = [](const JobDev& d) { return (d.ndim * 8 + vt::label_variant(d)) * 4 + d.cfg; };
    order.resize(n);
    for (int i = 0; i < n; ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(tab[a]) < key(tab[b]); });
    std::vector<JobDev> sorted((size_t)n);
    for (int k = 0; k < n; ++k)
        sorted[k] = tab[order[k]];
    tab.swap(sorted);
    groups.clear();
    group_of.assign(n, 0);
    int64_t ovf = 0;
    for (int k = 0; k < n;) {
        Group g{k, 0, vt::label_variant(tab[k]), tab[k].ndim, tab[k].cfg, 0, ovf};
        int kk = k;
        while (kk < n && key(tab[kk]) == key(tab[k])) {
            tab[kk].region_begin = g.regions;
            g.regions += tab[kk].nregions;
            group_of[kk] = (int)groups.size();
            ++kk;
        }
        g.count = kk - k;
        ovf += g.regions * 4;
        groups.push_back(g);
        k = kk;
    }
}

vt_status launch_groups(const JobDev* djobs, const std::vector<Group>& groups, int32_t* ovf_counts,
                        int32_t* ovf_list, hipStream_t s)
{
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group& g = groups[gi];
        VT_HIP(vt::launch_label_group(djobs + g.first, g.count, g.variant, g.ndim, g.cfg, g.regions,
                                      ovf_list + g.ovf_off, ovf_counts + gi, s));
    }
    return VT_OK;
}

}  // namespace

extern "C" {

const char* vt_status_string(vt_status s)
{
    switch (s) {
    case VT_OK: return "ok";
    case VT_ERR_INVALID: return "invalid argument";
    case VT_ERR_NOMEM: return "out of memory";
    case VT_ERR_HIP: return "HIP runtime error";
    case VT_ERR_BUSY: return "resource limit exceeded";
    case VT_ERR_INPUT: return "bad site data";
    }
    return "unknown status";
}

const char* vt_last_error(void) { return g_last_error.c_str(); }

vt_status vt_create(int device, vt_ctx** out)
{
    if (!out)
        return fail(VT_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    VT_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(VT_ERR_INVALID, "no such device");
    VT_HIP(hipSetDevice(device));
    vt_ctx* c = new vt_ctx();
    c->device = device;
    if (hipEventCreateWithFlags(&c->staging_evt, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return fail(VT_ERR_HIP, "event creation failed");
    }
    {
        // Once per device, with that device current: the address of this
        // device's copy of `scratch`.
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (device < kMaxDevices && !g_noalloc_ptr[device]) {
            void* p = nullptr;
            hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                (void)hipEventDestroy(c->staging_evt);
                delete c;
                return e != hipSuccess ? hip_fail(e, "hipGetSymbolAddress(scratch)")
                                       : fail(VT_ERR_HIP, "hipGetSymbolAddress(scratch) gave a null address");
            }
            g_noalloc_ptr[device] = p;
        }
        c->noalloc = device < kMaxDevices ? g_noalloc_ptr[device] : nullptr;
    }
    if (const char* path = std::getenv("VT_TUNE_CACHE"))
        vt_load_tuning(c, path);  // a missing cache is not an error
    *out = c;
    return VT_OK;
}

void vt_destroy(vt_ctx* ctx)
{
    if (!ctx)
        return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->arena)
        (void)hipFree(ctx->arena);
    if (ctx->pinned)
        (void)hipHostFree(ctx->pinned);
    if (ctx->staging_evt)
        (void)hipEventDestroy(ctx->staging_evt);
    for (hipEvent_t e : ctx->prof_events)
        (void)hipEventDestroy(e);
    delete ctx;
}

vt_status vt_set_params(vt_ctx* ctx, int32_t tile_cfg, double bin_factor)
{
    if (!ctx)
        return fail(VT_ERR_INVALID, "ctx is NULL");
    if (tile_cfg >= vt::kNumCfg)
        return fail(VT_ERR_INVALID, "tile_cfg must be 0, 1, 2 or 3 (or < 0)");
    if (!(bin_factor <= 0.0 || (bin_factor >= 0.125 && bin_factor <= 16.0)))
        return fail(VT_ERR_INVALID, "bin_factor out of range");
    ctx->force_cfg = tile_cfg;
    ctx->force_bin = bin_factor > 0.0 ? bin_factor : 0.0;
    return VT_OK;
}

vt_status vt_plan(vt_ctx* ctx, const vt_job* job, int32_t* bins_per_axis3, int32_t* tile_cfg, double* bin_factor)
{
    JobDev d;
    vt_status st = plan_job(ctx, job, &d);
    if (st != VT_OK)
        return st;
    if (bins_per_axis3)
        for (int a = 0; a < 3; ++a)
            bins_per_axis3[a] = d.nb[a];
    if (tile_cfg)
        *tile_cfg = d.cfg;
    if (bin_factor) {
        int cfg;
        choose_params(ctx, job, d.nvox, &cfg, bin_factor);
    }
    return VT_OK;
}

vt_status vt_tessellate(vt_ctx* ctx, const vt_job* job, int32_t* status_dev, void* stream)
{
    if (!ctx)
        return fail(VT_ERR_INVALID, "ctx is NULL");
    hipStream_t s = (hipStream_t)stream;
    JobDev d;
    vt_status st = plan_job(ctx, job, &d);
    if (st != VT_OK)
        return st;
    VT_HIP(hipSetDevice(ctx->device));
    const size_t zbytes = slot_layout(d).bytes;
    slots_for(ctx, 0, zbytes);
    const SingleLayout L = single_layout(d, ctx->slot_cap, 3);
    if ((st = ensure_scratch(ctx, L.total)) != VT_OK)
        return st;
    const SlotUse u = slot_begin(ctx, zbytes, s);
    const int slot = u.slot;
    const bool zeroed = u.zeroed, capturing = u.capturing;
    char* base = (char*)ctx->arena;
    bind_single(d, base, L, slot, status_dev);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (ctx->profile) {
        while (ctx->prof_events.size() < ctx->prof_used + 4) {
            hipEvent_t e;
            VT_HIP(hipEventCreate(&e));
            ctx->prof_events.push_back(e);
        }
        for (int k = 0; k < 4; ++k)
            ev[k] = ctx->prof_events[ctx->prof_used + k];
        ctx->prof_used += 4;
        VT_HIP(hipEventRecord(ev[0], s));
    }
    if ((st = bin_single(d, base, L, slot, zeroed, !capturing, s)) != VT_OK)
        return st;
    if (ev[1])
        VT_HIP(hipEventRecord(ev[1], s));
    const JobDev* jd = (const JobDev*)(base + L.job);
    VT_HIP(vt::launch_label_single(d, jd, s));
    if (ev[2])
        VT_HIP(hipEventRecord(ev[2], s));
    VT_HIP(vt::launch_label_fallback(d, jd, s));
    if (ev[3])
        VT_HIP(hipEventRecord(ev[3], s));
    slot_end(ctx, u, zbytes);
    return VT_OK;
}

vt_status vt_tessellate_noalloc(vt_ctx* ctx, const vt_job* job, int32_t* status_dev, void* stream)
{
    if (!ctx)
        return fail(VT_ERR_INVALID, "ctx is NULL");
    if (!ctx->noalloc)
        return fail(VT_ERR_HIP, "the static scratch is not set up on this device");
    hipStream_t s = (hipStream_t)stream;
    JobDev d;
    vt_status st = plan_job(ctx, job, &d);
    if (st != VT_OK)
        return st;
    const SingleLayout L = single_layout(d, slot_layout(d).bytes, 1);
    if (L.total > kNoallocBytes)
        return fail(VT_ERR_BUSY, "job needs " + std::to_string(L.total) +
                                     " bytes of scratch; vt_tessellate_noalloc has " +
                                     std::to_string(kNoallocBytes) + " (use vt_tessellate)");
    VT_HIP(hipSetDevice(ctx->device));
    // The same kernels as vt_tessellate on the device's static scratch; the
    // first binning kernel clears the counters and bounds that start at zero.
    char* base = (char*)ctx->noalloc;
    bind_single(d, base, L, 0, status_dev);
    if ((st = bin_single(d, base, L, 0, false, false, s)) != VT_OK)
        return st;
    VT_HIP(vt::launch_label_single(d, (const JobDev*)(base + L.job), s));
    VT_HIP(vt::launch_label_fallback(d, (const JobDev*)(base + L.job), s));
    return VT_OK;
}

// ---- general dimension ----

namespace {

// Inverse of the period matrix (columns = period vectors; Pinv[i][a] is
// fractional coordinate i per Cartesian axis a) by Gauss-Jordan elimination
// with partial pivoting; *det gets the determinant.  Used only for binning
// and bounds, so its rounding never reaches a key.  False when singular.
bool invert_periods(int d, const double* periods, double Pinv[vt::kMaxDim][vt::kMaxDim], double* det)
{
    double A[vt::kMaxDim][2 * vt::kMaxDim];
    double scale = 0.0;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            A[r][c] = periods[c * d + r];  // row r = Cartesian axis, column c = period vector
            A[r][d + c] = r == c ? 1.0 : 0.0;
            scale = std::max(scale, std::fabs(A[r][c]));
        }
    if (!(scale > 0.0))
        return false;
    double dt = 1.0;
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int r = c + 1; r < d; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c]))
                piv = r;
        if (!(std::fabs(A[piv][c]) > 1e-12 * scale))
            return false;
        if (piv != c) {
            for (int k = 0; k < 2 * d; ++k)
                std::swap(A[c][k], A[piv][k]);
            dt = -dt;
        }
        const double f = A[c][c];
        dt *= f;
        for (int k = 0; k < 2 * d; ++k)
            A[c][k] /= f;
        for (int r = 0; r < d; ++r) {
            if (r == c)
                continue;
            const double g = A[r][c];
            for (int k = 0; k < 2 * d; ++k)
                A[r][k] -= g * A[c][k];
        }
    }
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            Pinv[r][c] = A[r][d + c];
    *det = dt;
    return true;
}

// Tile shape of the general kernel: powers of two per axis, at most 256
// voxels, grown along the axis with the most voxels per tile side.
void nd_tile_shape(const vt_job_nd* j, int32_t* T)
{
    int prod = 1;
    for (int a = 0; a < j->ndim; ++a)
        T[a] = 1;
    while (prod * 2 <= 256) {
        int best = -1;
        double ratio = 1.0;
        for (int a = 0; a < j->ndim; ++a) {
            const double r = (double)j->n[a] / (double)T[a];
            if (T[a] < j->n[a] && r > ratio) {
                ratio = r;
                best = a;
            }
        }
        if (best < 0)
            break;
        T[best] *= 2;
        prod *= 2;
    }
}

// Squared length of the longest diagonal of the parallelepiped spanned by
// T[i] voxel steps d.hv[i] (i < nd).
double tile_diagonal2(const vt::NdDev& d, int nd, const int32_t* T)
{
    double worst = 0.0;
    for (int m = 0; m < (1 << (nd - 1)); ++m) {
        double q = 0.0;
        for (int a = 0; a < nd; ++a) {
            double x = 0.0;
            for (int i = 0; i < nd; ++i)
                x += ((i > 0 && ((m >> (i - 1)) & 1)) ? -1.0 : 1.0) * (double)T[i] * d.hv[i][a];
            q += x * x;
        }
        worst = std::max(worst, q);
    }
    return worst;
}

void lattice_shapes(const vt::NdDev& d, int nd, int axis, int left, const int* cap, int32_t* cur, int32_t* best,
                    double* bestd)
{
    if (axis == nd - 1) {
        if (left > cap[axis])
            return;
        cur[axis] = 1 << left;
        const double q = tile_diagonal2(d, nd, cur);
        if (q < *bestd) {
            *bestd = q;
            for (int a = 0; a < nd; ++a)
                best[a] = cur[a];
        }
        return;
    }
    for (int e = std::min(left, cap[axis]); e >= 0; --e) {
        cur[axis] = 1 << e;
        lattice_shapes(d, nd, axis + 1, left - e, cap, cur, best, bestd);
    }
}

// Tile shape with general period vectors (d.hv set): the first axis keeps
// the extent nd_tile_shape gives it; the others take, among the power-of-two
// shapes with as many voxels (each at most the smallest power of two not
// below its voxel count), the one whose tile parallelepiped has the shortest
// longest diagonal, so that fewer sites lie near a tile.  Ties keep the
// shape nd_tile_shape gives.  On the 3D triclinic benchmark cell this turns
// 8x8x4 into 8x4x8 tiles: 2-4 % faster per call for every kind.
void lattice_tile_shape(const vt_job_nd* j, const vt::NdDev& d, int32_t* T)
{
    nd_tile_shape(j, T);
    const int nd = j->ndim;
    if (nd < 3)
        return;
    int left = 0, cap[vt::kMaxDim] = {0};
    for (int a = 1; a < nd; ++a) {
        int e = 0;
        while ((1 << e) < T[a])
            ++e;
        left += e;
        int c = 0;
        while ((int64_t)1 << c < j->n[a])
            ++c;
        cap[a] = c;
    }
    int32_t cur[vt::kMaxDim], best[vt::kMaxDim];
    for (int a = 0; a < nd; ++a)
        cur[a] = best[a] = T[a];
    double bestd = tile_diagonal2(d, nd, T);
    lattice_shapes(d, nd, 1, left, cap, cur, best, &bestd);
    for (int a = 0; a < nd; ++a)
        T[a] = best[a];
}

vt_status plan_nd(const vt_ctx* ctx, const vt_job_nd* j, vt::NdDev* d)
{
    if (!j)
        return fail(VT_ERR_INVALID, "job is NULL");
    if (j->ndim < 1 || j->ndim > VT_MAX_DIM)
        return fail(VT_ERR_INVALID, "ndim must be in [1, 6]");
    if (j->kind < VT_VORONOI || j->kind > VT_JOHNSON_MEHL)
        return fail(VT_ERR_INVALID, "unknown diagram kind");
    if (j->bc != VT_NONPERIODIC && j->bc != VT_PERIODIC)
        return fail(VT_ERR_INVALID, "unknown boundary mode");
    if (j->flags & ~VT_ND_GENERIC)
        return fail(VT_ERR_INVALID, "unknown flags");
    if (j->nsites < 1 || j->nsites > 0x7fffffffLL)
        return fail(VT_ERR_INVALID, "nsites must be in [1, 2^31-1]");
    if (!j->coords || !j->labels)
        return fail(VT_ERR_INVALID, "coords and labels must be device pointers");
    if (j->kind != VT_VORONOI && !j->param)
        return fail(VT_ERR_INVALID, "param is required for Laguerre and Johnson-Mehl");
    if (j->kind == VT_JOHNSON_MEHL && !in_scale(j->growth))
        return fail(VT_ERR_INVALID, "growth rate must lie in [2^-200, 2^200]");
    std::memset(d, 0, sizeof *d);
    d->ndim = j->ndim;
    d->kind = j->kind;
    d->bc = j->bc ? 1 : 0;
    double nvox = 1.0, V = 1.0;
    for (int a = 0; a < j->ndim; ++a) {
        if (j->n[a] < 1 || j->n[a] > (1 << 30))
            return fail(VT_ERR_INVALID, "n[a] must be in [1, 2^30]");
        if (!j->periods && !in_scale(j->L[a]))
            return fail(VT_ERR_INVALID, "L[a] must lie in [2^-200, 2^200]");
        d->n[a] = j->n[a];
        d->L[a] = j->L[a];
        d->h[a] = j->L[a] / (double)j->n[a];
        d->H[a] = 0.5 * j->L[a];
        nvox *= (double)j->n[a];
        V *= j->L[a];
    }
    if (nvox > 1099511627776.0)
        return fail(VT_ERR_INVALID, "more than 2^40 voxels");
    d->nsites = (int32_t)j->nsites;
    d->growth = j->kind == VT_JOHNSON_MEHL ? j->growth : 1.0;
    d->rgrowth = 1.0 / d->growth;
    d->jm_div = (j->kind == VT_JOHNSON_MEHL && !is_pow2_scale(d->growth)) ? 1 : 0;

    // General period vectors: bins and tile bounds in fractional
    // coordinates (period 1 per axis).
    double extent[VT_MAX_DIM];
    for (int a = 0; a < j->ndim; ++a)
        extent[a] = j->L[a];
    if (j->periods) {
        const int nd = j->ndim;
        if (!j->bc)
            return fail(VT_ERR_INVALID, "period vectors need periodic boundaries");
        for (int k = 0; k < nd * nd; ++k)
            if (!(std::fabs(j->periods[k]) <= VT_SCALE_MAX))
                return fail(VT_ERR_INVALID, "period vector entries must be finite, |entry| <= 2^200");
        for (int i = 0; i < nd; ++i) {
            double n2 = 0.0;
            for (int a = 0; a < nd; ++a)
                n2 += j->periods[i * nd + a] * j->periods[i * nd + a];
            if (!in_scale(std::sqrt(n2)))
                return fail(VT_ERR_INVALID, "period vector lengths must lie in [2^-200, 2^200]");
        }
        double det = 0.0;
        if (!invert_periods(nd, j->periods, d->Pinv, &det))
            return fail(VT_ERR_INVALID, "period vectors are linearly dependent");
        d->lattice = 1;
        d->cell_d = 0.0;
        for (int i = 0; i < nd; ++i) {
            double n2 = 0.0, r2 = 0.0;
            for (int a = 0; a < nd; ++a) {
                d->P[i][a] = j->periods[i * nd + a];
                d->hv[i][a] = d->P[i][a] / (double)j->n[i];
                n2 += d->P[i][a] * d->P[i][a];
                r2 += d->Pinv[i][a] * d->Pinv[i][a];
            }
            d->rown[i] = std::sqrt(r2);
            if (!std::isfinite(d->rown[i]))
                return fail(VT_ERR_INVALID, "period vectors are too close to linearly dependent");
            d->cell_d += std::sqrt(n2);
            extent[i] = std::sqrt(n2);
            d->L[i] = 1.0;
            d->H[i] = 0.5;
            d->h[i] = 1.0 / (double)j->n[i];
        }
        V = std::fabs(det);
    }

    // Bins: side ~ 1.4 mean site spacings (V / N)^(1/d) with orthogonal
    // periods (or none) in 2 to 4 axes, else 1.2, or the bin factor
    // vt_set_params forces; at most 2^20 per axis and about 4 N + 64 in total.
    // Measured against 1.0 to 1.6 with the balanced search: 1.4 is 6-8 %
    // faster than 1.2 in 4D (64^4 Voronoi 1.04 -> 0.95 ms; Laguerre and
    // Johnson-Mehl 48^4) and for 3D through the general kernel; 5D is best
    // at 1.2 (1.62 against 1.73 ms), 6D and the triclinic cell are level.
    const double bin_factor = ctx && ctx->force_bin > 0.0       ? ctx->force_bin
                              : (!d->lattice && j->ndim >= 2 && j->ndim <= 4) ? 1.4
                                                                              : 1.2;
    const double spacing = std::pow(V / (double)j->nsites, 1.0 / j->ndim) * bin_factor;
    int64_t nbins = 1;
    for (int a = 0; a < j->ndim; ++a) {
        const double f = std::floor(extent[a] / spacing + 0.5);
        d->nb[a] = (int)std::min(std::max(f, 1.0), (double)(1 << 20));
        nbins *= d->nb[a];
    }
    const int64_t cap = std::min<int64_t>(4 * (int64_t)j->nsites + 64, (int64_t)1 << 28);
    while (nbins > cap) {
        nbins = 1;
        for (int a = 0; a < j->ndim; ++a) {
            d->nb[a] = std::max(1, d->nb[a] * 3 / 4);
            nbins *= d->nb[a];
        }
    }
    d->nbins = (int32_t)nbins;
    for (int a = 0; a < j->ndim; ++a) {
        d->bs[a] = d->L[a] / (double)d->nb[a];
        d->inv_bs[a] = (double)d->nb[a] / d->L[a];
    }
    if (d->lattice)
        lattice_tile_shape(j, *d, d->T);
    else
        nd_tile_shape(j, d->T);
    // Two voxels per thread along axis 0, so that a tile's search and staging
    // serve twice the voxels.  Measured to pay with orthogonal periods in 2 to
    // 4 axes when axis 0 holds at least eight thread widths (ragged tiles
    // waste little) and the doubled tiles still number 8,192 or more.  General
    // periods run a translation box per voxel, and 1, 5 and 6 axes, or fewer
    // tiles, came out slower.
    // (Four voxels per thread, under the same rule one step further, measured
    // twice as slow in 4D.)
    {
        int64_t tiles2 = 1;
        for (int a = 0; a < j->ndim; ++a) {
            const int64_t t = a == 0 ? 2 * (int64_t)d->T[0] : (int64_t)d->T[a];
            tiles2 *= (j->n[a] + t - 1) / t;
        }
        const bool two = !d->lattice && j->ndim >= 2 && j->ndim <= 4 && j->n[0] >= 8 * (int64_t)d->T[0] &&
                         tiles2 >= 8192;
        d->vpt = two ? 2 : 1;
    }
    d->T[0] *= d->vpt;
    d->ntiles = 1;
    for (int a = 0; a < j->ndim; ++a) {
        d->nt[a] = (j->n[a] + d->T[a] - 1) / d->T[a];
        d->ntiles *= d->nt[a];
    }
    d->coords = j->coords;
    d->param = j->param;
    d->labels = j->labels;
    d->keys = j->keys;
    return VT_OK;
}

}  // namespace

vt_status vt_plan_nd(vt_ctx* ctx, const vt_job_nd* job, int32_t* bins_per_axis, int32_t* tile_voxels)
{
    vt::NdDev d;
    vt_status st = plan_nd(ctx, job, &d);
    if (st != VT_OK)
        return st;
    for (int a = 0; a < job->ndim; ++a) {
        if (bins_per_axis)
            bins_per_axis[a] = d.nb[a];
        if (tile_voxels)
            tile_voxels[a] = d.T[a];
    }
    return VT_OK;
}

vt_status vt_tessellate_nd(vt_ctx* ctx, const vt_job_nd* job, int32_t* status_dev, void* stream)
{
    if (!ctx)
        return fail(VT_ERR_INVALID, "ctx is NULL");
    if (job && (job->ndim == 2 || job->ndim == 3) && !(job->flags & VT_ND_GENERIC) && !job->periods) {
        if (job->flags & ~VT_ND_GENERIC)
            return fail(VT_ERR_INVALID, "unknown flags");
        vt_job j;
        std::memset(&j, 0, sizeof j);
        j.ndim = job->ndim;
        j.kind = job->kind;
        j.bc = job->bc;
        for (int a = 0; a < job->ndim; ++a) {
            j.n[a] = job->n[a];
            j.L[a] = job->L[a];
        }
        j.growth = job->growth;
        j.nsites = job->nsites;
        j.coords = job->coords;
        j.param = job->param;
        j.labels = job->labels;
        j.keys = job->keys;
        return vt_tessellate(ctx, &j, status_dev, stream);
    }
    hipStream_t s = (hipStream_t)stream;
    vt::NdDev d;
    vt_status st = plan_nd(ctx, job, &d);
    if (st != VT_OK)
        return st;
    VT_HIP(hipSetDevice(ctx->device));
    // the words that start at zero: bounds, status accumulator, bin counts
    // (padded for the one-workgroup scan), flags of the multi-workgroup scan
    Carver z;
    const size_t z_pbound = z.take<unsigned long long>(3);
    const size_t z_sacc = z.take<int32_t>(1, 4);
    const size_t z_count = z.take<int32_t>(vt::count_words(d.nbins));
    const int64_t partial_cap = vt::scan_flags_needed((int64_t)d.nbins);
    const size_t z_partial = z.take<unsigned long long>(partial_cap, 8);
    const size_t zbytes = align_up(z.off, 256);
    slots_for(ctx, 1, zbytes);
    Carver c;
    size_t o_slot[3];
    for (int k = 0; k < 3; ++k)
        o_slot[k] = c.take<char>((int64_t)ctx->slot_cap);
    const size_t o_status = c.take<int32_t>(1, 4);
    const size_t o_start = c.take<int32_t>(vt::count_words(d.nbins) + 1);
    const size_t o_bin = c.take<int32_t>(d.nsites);
    const size_t o_rank = c.take<int32_t>(d.nsites);
    const size_t o_sc = c.take<double>((int64_t)d.nsites * d.ndim);
    const size_t o_sf = c.take<double>(d.lattice ? (int64_t)d.nsites * d.ndim : 0);
    const size_t o_sp = c.take<double>(d.nsites);
    const size_t o_sidx = c.take<int32_t>(d.nsites);
    if ((st = ensure_scratch(ctx, align_up(c.off, 256))) != VT_OK)
        return st;
    const SlotUse u = slot_begin(ctx, zbytes, s);
    char* base = (char*)ctx->arena;
    char* zs = base + o_slot[u.slot];
    d.pbound = (unsigned long long*)(zs + z_pbound);
    d.status = status_dev ? status_dev : (int32_t*)(base + o_status);
    d.bin_count = (int32_t*)(zs + z_count);
    d.bin_start = (int32_t*)(base + o_start);
    d.site_bin = (int32_t*)(base + o_bin);
    d.site_rank = (int32_t*)(base + o_rank);
    d.sc = (double*)(base + o_sc);
    d.sf = d.lattice ? (double*)(base + o_sf) : nullptr;
    d.sp = (double*)(base + o_sp);
    d.sidx = (int32_t*)(base + o_sidx);
    int32_t* sacc = (int32_t*)(zs + z_sacc);
    if (!u.zeroed)
        VT_HIP(launch_prepare((int32_t*)zs, (int64_t)(zbytes / 4), nullptr, s));
    int32_t* clear = u.capturing ? nullptr : (int32_t*)(base + o_slot[u.slot ^ 1]);
    VT_HIP(vt::launch_nd_bin_count(d, sacc, clear, clear ? (int64_t)(zbytes / 4) : 0, s));
    if (d.nbins <= vt::kSmallScanMax)
        VT_HIP(vt::launch_scan_small(d.bin_count, d.bin_start, d.nbins, s));
    else
        VT_HIP(vt::launch_scan(d.bin_count, d.bin_start, d.nbins, (unsigned long long*)(zs + z_partial), partial_cap,
                               s));
    VT_HIP(vt::launch_nd_bin_scatter(d, sacc, s));
    VT_HIP(vt::launch_nd_label(d, s));
    slot_end(ctx, u, zbytes);
    return VT_OK;
}

vt_status vt_profile_enable(vt_ctx* ctx, int32_t enable)
{
    if (!ctx)
        return fail(VT_ERR_INVALID, "ctx is NULL");
    ctx->profile = enable != 0;
    return VT_OK;
}

vt_status vt_profile_read(vt_ctx* ctx, double* bin_ms, double* label_ms, double* overflow_ms, int64_t* calls)
{
    if (!ctx)
        return fail(VT_ERR_INVALID, "ctx is NULL");
    double t[3] = {0.0, 0.0, 0.0};
    for (size_t k = 0; k + 4 <= ctx->prof_used; k += 4) {
        VT_HIP(hipEventSynchronize(ctx->prof_events[k + 3]));
        for (int p = 0; p < 3; ++p) {
            float ms = 0.0f;
            VT_HIP(hipEventElapsedTime(&ms, ctx->prof_events[k + p], ctx->prof_events[k + p + 1]));
            t[p] += ms;
        }
    }
    if (bin_ms)
        *bin_ms = t[0];
    if (label_ms)
        *label_ms = t[1];
    if (overflow_ms)
        *overflow_ms = t[2];
    if (calls)
        *calls = (int64_t)(ctx->prof_used / 4);
    ctx->prof_used = 0;
    return VT_OK;
}

vt_status vt_reserve(vt_ctx* ctx, size_t bytes)
{
    if (!ctx)
        return fail(VT_ERR_INVALID, "ctx is NULL");
    VT_HIP(hipSetDevice(ctx->device));
    return ensure_scratch(ctx, bytes);
}

vt_status vt_tessellate_batch(vt_ctx* ctx, const vt_job* jobs, int32_t njobs, int32_t* status_dev, void* stream)
{
    if (!ctx)
        return fail(VT_ERR_INVALID, "ctx is NULL");
    if (njobs < 1 || !jobs)
        return fail(VT_ERR_INVALID, "need at least one job");
    hipStream_t s = (hipStream_t)stream;
    std::vector<JobDev> host((size_t)njobs);
    for (int i = 0; i < njobs; ++i) {
        vt_status st = plan_job(ctx, &jobs[i], &host[i]);
        if (st != VT_OK)
            return fail(st, "job " + std::to_string(i) + ": " + g_last_error);
    }
    std::vector<int> order, group_of;
    std::vector<Group> groups;
    make_groups(host, order, group_of, groups);
    const int ng = (int)groups.size();
    std::vector<int64_t> prefix((size_t)njobs + 1, 0);
    int64_t total_bins = 0, total_tiles = 0;
    for (int k = 0; k < njobs; ++k) {
        prefix[k + 1] = prefix[k] + host[k].nsites;
        host[k].site_begin = prefix[k];
        host[k].bin_begin = total_bins;
        total_tiles += host[k].nregions;
        total_bins += host[k].nbins;
    }
    const int64_t total_sites = prefix[njobs];
    if (total_sites > 0x7fffffffLL || total_bins > 0x7ffffffeLL)
        return fail(VT_ERR_BUSY, "batch too large: more than 2^31 sites or bins");
    VT_HIP(hipSetDevice(ctx->device));
    // Layout: [pbound 2/job][status 1/job][bin_count][overflow count 1/group]
    // [scan flags] zeroed together, then bin_start, site arrays, overflow
    // lists.
    Carver c;
    const size_t o_pb = c.take<unsigned long long>(2 * (int64_t)njobs);
    const size_t o_st = c.take<int32_t>(njobs, 8);
    const size_t o_cnt = c.take<int32_t>(vt::count_words(total_bins));  // padded for the one-workgroup scan
    const size_t o_ovfc = c.take<int32_t>(ng, 4);
    const int64_t pcap = vt::scan_flags_needed(total_bins);
    const size_t o_part = c.take<unsigned long long>(pcap, 8);  // scan flags, cleared with the counts
    const size_t zero_end = c.off;
    const size_t o_start = c.take<int32_t>(vt::count_words(total_bins) + 1);
    const size_t o_sbin = c.take<int32_t>(total_sites);
    const size_t o_srank = c.take<int32_t>(total_sites);
    const size_t o_sites = c.take<double4>(total_sites);
    const size_t o_sidx = c.take<int32_t>(total_sites);
    const size_t o_ovf = c.take<int32_t>(total_tiles * 4);
    const size_t jb = align_up(host.size() * sizeof(JobDev), 256);
    const size_t o_tab = c.take<char>((int64_t)(jb + prefix.size() * sizeof(int64_t)), 256);
    vt_status st = ensure_scratch(ctx, align_up(c.off, 256));
    if (st != VT_OK)
        return st;
    ctx->slot_owner = -1;  // the arena's words are reused below
    ctx->slot_clean[0] = ctx->slot_clean[1] = 0;
    char* base = (char*)ctx->arena;
    for (int k = 0; k < njobs; ++k) {
        JobDev& d = host[k];
        const Group& g = groups[group_of[k]];
        d.pbound = (unsigned long long*)(base + o_pb) + 2 * k;
        d.status = status_dev ? status_dev + order[k] : (int32_t*)(base + o_st) + k;
        d.bin_count = (int32_t*)(base + o_cnt) + d.bin_begin;
        d.bin_start = (int32_t*)(base + o_start) + d.bin_begin;  // values index the batch-wide site arrays
        d.site_bin = (int32_t*)(base + o_sbin) + prefix[k];
        d.site_rank = (int32_t*)(base + o_srank) + prefix[k];
        d.sites = (double4*)(base + o_sites);
        d.sidx = (int32_t*)(base + o_sidx);
        d.ovf_count = (int32_t*)(base + o_ovfc) + group_of[k];
        d.ovf_list = (int32_t*)(base + o_ovf) + g.ovf_off;
    }
    // job table and site prefix, in the scratch arena (stream-ordered like the
    // rest of it)
    std::vector<char> blob(jb + prefix.size() * sizeof(int64_t));
    std::memcpy(blob.data(), host.data(), host.size() * sizeof(JobDev));
    std::memcpy(blob.data() + jb, prefix.data(), prefix.size() * sizeof(int64_t));
    void* table = base + o_tab;
    if ((st = stage_copy(ctx, table, blob.data(), blob.size(), s)) != VT_OK)
        return st;
    const JobDev* djobs = (const JobDev*)table;
    const int64_t* dprefix = (const int64_t*)((char*)table + jb);
    VT_HIP(launch_prepare((int32_t*)(base + o_pb), (int64_t)((zero_end - o_pb) / 4), nullptr, s));
    if (status_dev)
        VT_HIP(vt::launch_fill_i32(status_dev, njobs, 0, s));
    JobDev dummy;
    std::memset(&dummy, 0, sizeof dummy);
    VT_HIP(vt::launch_bin_count(dummy, djobs, njobs, dprefix, total_sites, s));
    if (total_bins <= vt::kSmallScanMax)
        VT_HIP(vt::launch_scan_small((int32_t*)(base + o_cnt), (int32_t*)(base + o_start), total_bins, s));
    else
        VT_HIP(vt::launch_scan((int32_t*)(base + o_cnt), (int32_t*)(base + o_start), total_bins,
                               (unsigned long long*)(base + o_part), pcap, s));
    VT_HIP(vt::launch_bin_scatter(dummy, djobs, njobs, dprefix, total_sites, s));
    VT_HIP(vt::launch_jm_prune(dummy, djobs, njobs, dprefix, total_sites, total_bins, s));
    return launch_groups(djobs, groups, (int32_t*)(base + o_ovfc),
                         (int32_t*)(base + o_ovf), s);
}

vt_status vt_bins_build(vt_ctx* ctx, const vt_job* job, vt_bins** out, int32_t* status_dev, void* stream)
{
    if (!ctx || !out)
        return fail(VT_ERR_INVALID, "ctx and out must not be NULL");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    JobDev d;
    vt_status st = plan_job(ctx, job, &d);
    if (st != VT_OK)
        return st;
    VT_HIP(hipSetDevice(ctx->device));
    const SingleLayout L = single_layout(d, slot_layout(d).bytes, 1);
    void* mem = nullptr;
    if (hipMallocAsync(&mem, L.total, s) != hipSuccess)
        return fail(VT_ERR_NOMEM, "bins allocation failed");
    char* base = (char*)mem;
    bind_single(d, base, L, 0, nullptr);
    if ((st = bin_single(d, base, L, 0, false, false, s)) != VT_OK) {
        (void)hipFreeAsync(mem, s);
        return st;
    }
    if (status_dev)
        VT_HIP(hipMemcpyAsync(status_dev, d.status, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    vt_bins* b = new vt_bins();
    b->job = d;
    b->mem = mem;
    *out = b;
    return VT_OK;
}

vt_status vt_label_batch(vt_ctx* ctx, vt_bins* const* bins, int32_t n, int32_t* status_dev, void* stream)
{
    if (!ctx || !bins || n < 1)
        return fail(VT_ERR_INVALID, "need a context and at least one bins object");
    hipStream_t s = (hipStream_t)stream;
    std::vector<JobDev> host((size_t)n);
    for (int i = 0; i < n; ++i) {
        if (!bins[i])
            return fail(VT_ERR_INVALID, "bins[" + std::to_string(i) + "] is NULL");
        host[i] = bins[i]->job;
    }
    std::vector<int> order, group_of;
    std::vector<Group> groups;
    make_groups(host, order, group_of, groups);
    const int ng = (int)groups.size();
    int64_t total_tiles = 0;
    for (const JobDev& d : host)
        total_tiles += d.nregions;
    VT_HIP(hipSetDevice(ctx->device));
    // One stream-ordered allocation: job table, the caller's order, then one
    // overflow count per group (zeroed on the device), then the overflow lists.
    const size_t jb = align_up((size_t)n * sizeof(JobDev), 256);
    const size_t ob = align_up((size_t)n * sizeof(int32_t), 256);
    const size_t cb = align_up((size_t)ng * sizeof(int32_t), 256);
    const size_t bytes = jb + ob + cb + (size_t)total_tiles * 4 * sizeof(int32_t);
    void* table = nullptr;
    vt_status st = alloc_table(bytes, s, &table);
    if (st != VT_OK)
        return st;
    int32_t* dorder = (int32_t*)((char*)table + jb);
    int32_t* ovf_counts = (int32_t*)((char*)table + jb + ob);
    int32_t* ovf_list = (int32_t*)((char*)table + jb + ob + cb);
    for (int k = 0; k < n; ++k) {
        host[k].ovf_count = ovf_counts + group_of[k];
        host[k].ovf_list = ovf_list + groups[group_of[k]].ovf_off;
    }
    std::vector<char> blob(jb + ob);
    std::memcpy(blob.data(), host.data(), (size_t)n * sizeof(JobDev));
    std::memcpy(blob.data() + jb, order.data(), (size_t)n * sizeof(int32_t));
    if ((st = stage_copy(ctx, table, blob.data(), blob.size(), s)) != VT_OK)
        return st;
    VT_HIP(vt::launch_fill_i32(ovf_counts, ng, 0, s));
    const JobDev* djobs = (const JobDev*)table;
    if ((st = launch_groups(djobs, groups, ovf_counts, ovf_list, s)) != VT_OK)
        return st;
    if (status_dev)
        k_copy_status<<<(n + 255) / 256, 256, 0, s>>>(djobs, n, dorder, status_dev);
    VT_HIP(hipGetLastError());
    VT_HIP(hipFreeAsync(table, s));
    return VT_OK;
}

vt_status vt_bins_free(vt_ctx* ctx, vt_bins* bins, void* stream)
{
    if (!ctx)
        return fail(VT_ERR_INVALID, "ctx is NULL");
    if (!bins)
        return VT_OK;
    VT_HIP(hipSetDevice(ctx->device));
    hipError_t e = hipFreeAsync(bins->mem, (hipStream_t)stream);
    delete bins;
    if (e != hipSuccess)
        return hip_fail(e, "hipFreeAsync");
    return VT_OK;
}

constexpr unsigned long long kDigestP = 2147483647ull;  // 2^31 - 1

// x mod (2^31 - 1) for x < 2^63, by folding the bits above 31 (2^31 = 1 mod P).
__device__ inline unsigned long long mod_p31(unsigned long long x)
{
    x = (x & kDigestP) + (x >> 31);  // < 2^32 + 2^31
    x = (x & kDigestP) + (x >> 31);  // <= P + 3
    return x >= kDigestP ? x - kDigestP : x;
}

__global__ __launch_bounds__(256) void k_digest(const int32_t* __restrict__ lab, int64_t n,
                                                unsigned long long* acc)
{
    // Every product is below 2^62 and each partial sum is reduced after every
    // term, so unsigned 64-bit arithmetic is exact.
    __shared__ unsigned long long part[256 / 64];
    unsigned long long h = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        const unsigned long long w = mod_p31((unsigned long long)i * 48271ull + 97ull);
        const long long t = (long long)lab[i] + 3;  // any int32 label; the mod is the non-negative one
        const unsigned long long v = t >= 0 ? mod_p31((unsigned long long)t)
                                            : mod_p31(kDigestP - mod_p31((unsigned long long)(-t)));
        h = mod_p31(h + v * w);
    }
    for (int o = 32; o > 0; o >>= 1)
        h += __shfl_xor(h, o);  // 64 terms below 2^31: no wrap
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x / 64] = mod_p31(h);
    __syncthreads();
    if (threadIdx.x == 0)
        atomicAdd(acc, mod_p31(part[0] + part[1] + part[2] + part[3]));
}

vt_status vt_label_digest(vt_ctx* ctx, const int32_t* labels, int64_t n, unsigned long long* acc_dev, void* stream)
{
    if (!ctx || n < 0 || !acc_dev || (n > 0 && !labels))
        return fail(VT_ERR_INVALID, "bad digest arguments");
    if (n == 0)
        return VT_OK;
    VT_HIP(hipSetDevice(ctx->device));
    // A grid-stride launch of at most 1024 workgroups: each adds one partial
    // sum, so the accumulator sees few atomics.
    int64_t g = (n + 255) / 256;
    g = std::min<int64_t>(g, 1024);
    k_digest<<<(unsigned)g, 256, 0, (hipStream_t)stream>>>(labels, n, acc_dev);
    VT_HIP(hipGetLastError());
    return VT_OK;
}

vt_status vt_numerics_probe(vt_ctx* ctx, const double* x, const double* den, double* sqrt_out, double* div_out,
                            int64_t n, void* stream)
{
    if (!ctx || n < 0 || (n > 0 && (!x || !den || !sqrt_out || !div_out)))
        return fail(VT_ERR_INVALID, "bad probe arguments");
    if (n == 0)
        return VT_OK;
    VT_HIP(hipSetDevice(ctx->device));
    const int64_t g = (n + 255) / 256;
    if (g > 0x7fffffffLL)
        return fail(VT_ERR_INVALID, "probe too large");
    k_probe<<<(unsigned)g, 256, 0, (hipStream_t)stream>>>(x, den, sqrt_out, div_out, n);
    VT_HIP(hipGetLastError());
    return VT_OK;
}

vt_status vt_load_tuning(vt_ctx* ctx, const char* cache_path)
{
    if (!ctx || !cache_path)
        return fail(VT_ERR_INVALID, "ctx and cache_path must not be NULL");
    FILE* f = std::fopen(cache_path, "r");
    if (!f)
        return fail(VT_ERR_INVALID, std::string("cannot open ") + cache_path);
    char line[512];
    std::vector<TuneEntry> got;
    while (std::fgets(line, sizeof line, f)) {
        TuneEntry t;
        if (std::sscanf(line,
                        " {\"ndim\": %d, \"kind\": %d, \"bc\": %d, \"size_class\": %d, \"density_class\": %d, "
                        "\"tile_cfg\": %d, \"bin_factor\": %lf, \"gather_margin\": %d, \"ms\": %lf, "
                        "\"default_ms\": %lf",
                        &t.ndim, &t.kind, &t.bc, &t.size_cls, &t.dens_cls, &t.cfg, &t.bin_factor, &t.gather_margin,
                        &t.ms, &t.default_ms) == 10 &&
            t.cfg >= 0 && t.cfg < vt::kNumCfg && t.bin_factor >= 0.125 && t.bin_factor <= 16.0)
            got.push_back(t);
    }
    std::fclose(f);
    for (const TuneEntry& t : got) {
        bool replaced = false;
        for (TuneEntry& o : ctx->tune)
            if (o.ndim == t.ndim && o.kind == t.kind && o.bc == t.bc && o.size_cls == t.size_cls &&
                o.dens_cls == t.dens_cls) {
                o = t;
                replaced = true;
            }
        if (!replaced)
            ctx->tune.push_back(t);
    }
    return VT_OK;
}

}  // extern "C"

namespace {

// One tuning round over the samples of a class: each sample alone
// (vt_tessellate), then all of them in one vt_tessellate_batch call, so that
// the plan is judged on the single-job and the batch kernels; the best of
// three rounds after a warm-up.
vt_status time_round(vt_ctx* ctx, const std::vector<vt_job>& js, hipEvent_t e0, hipEvent_t e1, double* ms)
{
    vt_status st;
    for (const vt_job& j : js)
        if ((st = vt_tessellate(ctx, &j, nullptr, nullptr)) != VT_OK)
            return st;
    if ((st = vt_tessellate_batch(ctx, js.data(), (int32_t)js.size(), nullptr, nullptr)) != VT_OK)
        return st;
    float best = 1e30f;
    for (int r = 0; r < 3; ++r) {
        VT_HIP(hipEventRecord(e0, nullptr));
        for (const vt_job& j : js)
            if ((st = vt_tessellate(ctx, &j, nullptr, nullptr)) != VT_OK)
                return st;
        if ((st = vt_tessellate_batch(ctx, js.data(), (int32_t)js.size(), nullptr, nullptr)) != VT_OK)
            return st;
        VT_HIP(hipEventRecord(e1, nullptr));
        VT_HIP(hipEventSynchronize(e1));
        float t = 0.0f;
        VT_HIP(hipEventElapsedTime(&t, e0, e1));
        best = std::min(best, t);
    }
    *ms = best;
    return VT_OK;
}

vt_status tune_classes(vt_ctx* ctx, const vt_job* samples, int32_t n)
{
    // samples by class (dimension, kind, boundary, size class, density class)
    std::vector<std::vector<vt_job>> cls;
    std::vector<TuneEntry> keys;
    for (int i = 0; i < n; ++i) {
        JobDev d;
        vt_status st = plan_job(ctx, &samples[i], &d);
        if (st != VT_OK)
            return st;
        TuneEntry k{};
        k.ndim = samples[i].ndim;
        k.kind = samples[i].kind;
        k.bc = samples[i].bc ? 1 : 0;
        k.size_cls = size_class(d.nvox);
        k.dens_cls = dens_class(d.nvox, samples[i].nsites);
        size_t c = 0;
        while (c < keys.size() && !(keys[c].ndim == k.ndim && keys[c].kind == k.kind && keys[c].bc == k.bc &&
                                    keys[c].size_cls == k.size_cls && keys[c].dens_cls == k.dens_cls))
            ++c;
        if (c == keys.size()) {
            keys.push_back(k);
            cls.emplace_back();
        }
        cls[c].push_back(samples[i]);
    }
    hipEvent_t e0, e1;
    VT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(VT_ERR_HIP, "event creation failed");
    }
    // Tile configurations 0-3, bins of 1.0 to 2.0 mean spacings (every factor
    // the built-in plans use), and for Laguerre the first gather margin.
    const double factors[] = {1.0, 1.2, 1.4, 1.6, 2.0};
    vt_status st = VT_OK;
    for (size_t c = 0; c < cls.size() && st == VT_OK; ++c) {
        TuneEntry best = keys[c];
        // the built-in plan of this class, without the tuning table
        ctx->skip_tune = true;
        ctx->force_cfg = -1;
        ctx->force_bin = 0.0;
        ctx->force_margin = 0;
        double t_def = 0.0;
        if ((st = time_round(ctx, cls[c], e0, e1, &t_def)) != VT_OK)
            break;
        {
            JobDev d;
            if ((st = plan_job(ctx, &cls[c][0], &d)) != VT_OK)
                break;
            int cfg, margin;
            double bf;
            choose_params(ctx, &cls[c][0], d.nvox, &cfg, &bf, &margin);
            best.cfg = cfg;
            best.bin_factor = bf;
            best.gather_margin = margin;
        }
        best.ms = t_def;
        best.default_ms = t_def;
        const int nmargin = keys[c].kind == VT_LAGUERRE ? 2 : 1;
        for (int cfg = 0; cfg < vt::kNumCfg && st == VT_OK; ++cfg)
            for (double bf : factors)
                for (int m = 1; m <= nmargin && st == VT_OK; ++m) {
                    ctx->force_cfg = cfg;
                    ctx->force_bin = bf;
                    ctx->force_margin = nmargin > 1 ? m : 0;
                    double t = 0.0;
                    if ((st = time_round(ctx, cls[c], e0, e1, &t)) != VT_OK)
                        break;
                    // a candidate replaces the current best only when clearly
                    // faster, so that timing noise never trades a measured
                    // default for an equal plan
                    if (t < best.ms * 0.97) {
                        best.ms = t;
                        best.cfg = cfg;
                        best.bin_factor = bf;
                        best.gather_margin = nmargin > 1 ? m : 0;
                    }
                }
        if (st != VT_OK)
            break;
        bool replaced = false;
        for (TuneEntry& o : ctx->tune)
            if (o.ndim == best.ndim && o.kind == best.kind && o.bc == best.bc && o.size_cls == best.size_cls &&
                o.dens_cls == best.dens_cls) {
                o = best;
                replaced = true;
            }
        if (!replaced)
            ctx->tune.push_back(best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

extern "C" {

vt_status vt_autotune(vt_ctx* ctx, const vt_job* samples, int32_t n, const char* cache_path)
{
    if (!ctx || !samples || n < 1)
        return fail(VT_ERR_INVALID, "need a context and at least one sample job");
    VT_HIP(hipSetDevice(ctx->device));
    const int saved_cfg = ctx->force_cfg;
    const double saved_bin = ctx->force_bin;
    vt_status result = tune_classes(ctx, samples, n);
    ctx->force_cfg = saved_cfg;
    ctx->force_bin = saved_bin;
    ctx->force_margin = 0;
    ctx->skip_tune = false;
    if (result != VT_OK)
        return result;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "w");
        if (!f)
            return fail(VT_ERR_INVALID, std::string("cannot write ") + cache_path);
        std::fprintf(f, "[\n");
        for (size_t k = 0; k < ctx->tune.size(); ++k) {
            const TuneEntry& t = ctx->tune[k];
            std::fprintf(f,
                         " {\"ndim\": %d, \"kind\": %d, \"bc\": %d, \"size_class\": %d, \"density_class\": %d, "
                         "\"tile_cfg\": %d, \"bin_factor\": %.3f, \"gather_margin\": %d, \"ms\": %.6f, "
                         "\"default_ms\": %.6f}%s\n",
                         t.ndim, t.kind, t.bc, t.size_cls, t.dens_cls, t.cfg, t.bin_factor, t.gather_margin, t.ms,
                         t.default_ms, k + 1 < ctx->tune.size() ? "," : "");
        }
        std::fprintf(f, "]\n");
        std::fclose(f);
    }
    return VT_OK;
}

}  // extern "C"
