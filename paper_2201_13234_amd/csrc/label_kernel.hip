// label_kernel.hip -- per-voxel argmin of the diagram's key over the sites,
// one wavefront (64 lanes) per voxel tile.
//
// What is computed (Sec. 2, Sec. 3 problem statement, App. A): for every voxel
// centre x, the lowest index s minimising
//     Voronoi q,  Laguerre q - w_s,  Johnson-Mehl t_s + sqrt(q) / v,
// q = d0*d0 + (d1*d1 + d2*d2) with minimum-image differences for periodic
// boundaries, each operation rounded once in binary64 (build flags keep the
// compiler from contracting into fused multiply-add).
//
// How (our GPU design, not the paper's CPU ball scheme):
//   1. Gather.  Walk the uniform bin grid outward from the tile, one shell of
//      bins at a time.  Each gathered site gets a lower and an upper bound of
//      its key over the tile's box of voxel centres; UB = min over gathered
//      sites of their upper bound bounds every voxel's winning key.  Sites
//      whose lower bound exceeds UB are dropped at once.  The walk stops when
//      a lower bound of the key of every site outside the visited bins
//      (gap^2, gap^2 - max w, min t + gap / v) exceeds UB, or when every bin has
//      been visited.
//   2. Prune.  A site is dropped if another site beats it on the whole tile:
//      for Voronoi and Laguerre the key difference of two sites is linear in x,
//      so its minimum over the box is at a corner; for Johnson-Mehl a bound of
//      the difference of distances is used.
//   3. Sort the survivors by site index and evaluate them for every voxel of
//      the lane's run with the exact key and a strict '<' -- the paper's
//      brute-force loop restricted to the survivors, which gives the lowest
//      index on ties.
// Every bound test keeps a margin of 2^-36 times the problem's key scale, far
// above the rounding error of any computed key, so a dropped site's computed
// key is strictly larger than the winner's at every voxel of the tile: the
// labels equal brute force bit for bit.
#include "vt_internal.h"

namespace vt {

namespace {

struct WaveLds {
    double4 cs[CAP];   // candidate site {x, y, z, param}
    double2 cb[CAP];   // {lower, upper} bound of the key over the tile box
    double2 cq[CAP];   // {min, max} distance to the tile box
    int2 cm[CAP];      // {site index, flags}
    int bcnt[WAVE];    // inclusive prefix of site counts of the current bin chunk
    int bsrc[WAVE];    // first sorted-site position of each bin of the chunk
};

// flags: wrap code per axis in bits 2a..2a+1 (0 none, 1 subtract L, 2 add L),
// bit 6 = some axis needs a per-voxel minimum-image test.
constexpr int FL_GENERIC = 64;

enum { KV = 0, KL = 1, KJM = 2, KJD = 3 };  // Johnson-Mehl: multiply by exact 1/v, or divide

__device__ inline int wrap_code(double d, double H) { return d >= H ? 1 : (d < -H ? 2 : 0); }
__device__ inline double code_off(int c, double L) { return c == 1 ? -L : (c == 2 ? L : 0.0); }
__device__ inline double min_image(double d, double H, double L)
{
    return d >= H ? d - L : (d < -H ? d + L : d);
}

__device__ inline double from_ordered(unsigned long long u)
{
    unsigned long long b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)b);
}

__device__ inline double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmin(v, __shfl_xor(v, o));
    return v;
}

__device__ inline int wave_inclusive_add(int v, int lane)
{
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(v, o);
        if (lane >= o)
            v += t;
    }
    return v;
}

__device__ inline unsigned long long lanes_below(int lane)
{
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

template <int KIND>
__device__ inline double dist_key(double q, double p, double v, double rv)
{
    if (KIND == KV)
        return q;
    if (KIND == KL)
        return q - p;
    if (KIND == KJM)
        return p + sqrt(q) * rv;
    return p + sqrt(q) / v;
}

struct TileBox {
    double lo[3], hi[3];  // box of voxel centres
};

// Keeps the entries of the wave's list whose predicate holds, in order.
// keep0/keep1 refer to entries lane and lane + 64.
__device__ inline int compact(WaveLds& S, int nc, bool keep0, bool keep1, int lane)
{
    double4 s0, s1;
    double2 b0, b1, q0, q1;
    int2 m0, m1;
    const bool v0 = lane < nc, v1 = lane + WAVE < nc;
    keep0 = keep0 && v0;
    keep1 = keep1 && v1;
    if (v0) {
        s0 = S.cs[lane];
        b0 = S.cb[lane];
        q0 = S.cq[lane];
        m0 = S.cm[lane];
    }
    if (v1) {
        s1 = S.cs[lane + WAVE];
        b1 = S.cb[lane + WAVE];
        q1 = S.cq[lane + WAVE];
        m1 = S.cm[lane + WAVE];
    }
    __syncthreads();
    const unsigned long long k0 = __ballot(keep0), k1 = __ballot(keep1);
    const int n0 = __popcll(k0);
    if (keep0) {
        int d = __popcll(k0 & lanes_below(lane));
        S.cs[d] = s0;
        S.cb[d] = b0;
        S.cq[d] = q0;
        S.cm[d] = m0;
    }
    if (keep1) {
        int d = n0 + __popcll(k1 & lanes_below(lane));
        S.cs[d] = s1;
        S.cb[d] = b1;
        S.cq[d] = q1;
        S.cm[d] = m1;
    }
    __syncthreads();
    return n0 + __popcll(k1);
}

// True if site c (entry e) loses to some other listed site on the whole box.
template <int KIND, int DIM>
__device__ inline bool dominated(const WaveLds& S, int nc, int e, const JobDev& J, const TileBox& B,
                                 double M, double sumL2_sqrt, double rv)
{
    const double4 c = S.cs[e];
    const int2 cm = S.cm[e];
    const double2 cq = S.cq[e];
    const double2 cb = S.cb[e];
    const bool cgen = (cm.y & FL_GENERIC) != 0;
    double sc[3] = {c.x, c.y, c.z};
    if (!cgen)
        for (int a = 0; a < DIM; ++a)
            sc[a] += code_off((cm.y >> (2 * a)) & 3, J.L[a]);
    bool dom = false;
    for (int t = 0; t < nc; ++t) {
        if (t == e)
            continue;
        const double4 o = S.cs[t];
        const int2 om = S.cm[t];
        if (KIND == KV || KIND == KL) {
            if (cgen || (om.y & FL_GENERIC))
                continue;
            // key_c - key_t = sum_a (sc - so)(sc + so - 2 x_a) - w_c + w_t, linear in x
            double so[3] = {o.x, o.y, o.z};
            double D = 0.0;
            for (int a = 0; a < DIM; ++a) {
                so[a] += code_off((om.y >> (2 * a)) & 3, J.L[a]);
                double al = sc[a] - so[a];
                double xs = al > 0.0 ? B.hi[a] : B.lo[a];
                D += al * ((sc[a] + so[a]) - 2.0 * xs);
            }
            if (KIND == KL)
                D = D - c.w + o.w;
            if (D > M)
                dom = true;
        } else {
            // t_c + d_c/v - (t_t + d_t/v) >= (t_c - t_t) + lbd / v, lbd a lower
            // bound of d_c - d_t over the box.
            const double2 oq = S.cq[t];
            double lbd = cq.x - oq.y;
            if (!cgen && !(om.y & FL_GENERIC)) {
                double Dq = 0.0;
                for (int a = 0; a < DIM; ++a) {
                    double so = (a == 0 ? o.x : (a == 1 ? o.y : o.z)) +
                                code_off((om.y >> (2 * a)) & 3, J.L[a]);
                    double al = sc[a] - so;
                    double xs = al > 0.0 ? B.hi[a] : B.lo[a];
                    Dq += al * ((sc[a] + so) - 2.0 * xs);
                }
                const double floor_den = sumL2_sqrt * 0x1p-10;
                if (Dq > 0.0) {
                    double den = cq.y + oq.y;
                    if (den >= floor_den)
                        lbd = fmax(lbd, Dq / den);
                } else {
                    double den = cq.x + oq.x;
                    if (den >= floor_den)
                        lbd = fmax(lbd, Dq / den);
                }
            }
            double f = (c.w - o.w) + lbd * rv;
            if (f > M)
                dom = true;
        }
        (void)cb;
    }
    return dom;
}

template <int KIND, int DIM, int RUN, int LX, int LY, int LZ>
__device__ void label_tile(const JobDev& J, int64_t tile, WaveLds& S, const int lane)
{
    constexpr int TX = RUN * LX, TY = LY, TZ = (DIM == 3) ? LZ : 1;
    static_assert(LX * LY * LZ == WAVE, "64 lanes per tile");
    const bool periodic = J.bc != 0;

    // ---- tile and lane geometry
    const int tx = (int)(tile % J.nt[0]);
    const int64_t rr = tile / J.nt[0];
    const int ty = (int)(rr % J.nt[1]);
    const int tz = (int)(rr / J.nt[1]);
    const int v0[3] = {tx * TX, ty * TY, tz * TZ};
    const int ve[3] = {min(v0[0] + TX, J.n[0]) - 1, min(v0[1] + TY, J.n[1]) - 1,
                       min(v0[2] + TZ, J.n[2]) - 1};
    TileBox B;
    for (int a = 0; a < 3; ++a) {
        if (a < DIM) {
            B.lo[a] = ((double)v0[a] + 0.5) * J.h[a];
            B.hi[a] = ((double)ve[a] + 0.5) * J.h[a];
        } else {
            B.lo[a] = B.hi[a] = 0.0;
        }
    }
    const int lx = lane % LX, ly = (lane / LX) % LY, lz = lane / (LX * LY);
    const int mi = v0[0] + lx * RUN, mj = v0[1] + ly, mk = (DIM == 3) ? v0[2] + lz : 0;
    double xr[RUN];
#pragma unroll
    for (int q = 0; q < RUN; ++q)
        xr[q] = ((double)(mi + q) + 0.5) * J.h[0];
    const double yv = ((double)mj + 0.5) * J.h[1];
    const double zv = (DIM == 3) ? ((double)mk + 0.5) * J.h[2] : 0.0;
    double best[RUN];
    int lab[RUN];
#pragma unroll
    for (int q = 0; q < RUN; ++q) {
        best[q] = __builtin_inf();
        lab[q] = -1;
    }

    const bool bad = *(volatile int32_t*)J.status != 0;
    if (!bad) {
        // ---- per-job constants: key scale, margin, bounds of the parameters
        double sumL2 = 0.0;
        for (int a = 0; a < DIM; ++a)
            sumL2 += J.L[a] * J.L[a];
        const double sumL2_sqrt = sqrt(sumL2);
        const double v = J.growth, rv = J.rgrowth;
        double pmax = 0.0, pmin = 0.0;
        if (KIND != KV) {
            pmax = from_ordered(J.pbound[0]);
            pmin = -from_ordered(J.pbound[1]);
        }
        const double pabs = fmax(fabs(pmax), fabs(pmin));
        const double scale = (KIND == KV) ? sumL2
                             : (KIND == KL) ? sumL2 + 2.0 * pabs
                                            : sumL2_sqrt * rv + 2.0 * pabs;
        const double M = scale * 0x1p-36;

        // ---- visited bin box (unwrapped bin coordinates) and previous box
        int blo[3], bhi[3], olo[3], ohi[3];
        for (int a = 0; a < 3; ++a) {
            if (a < DIM) {
                int l = (int)(B.lo[a] * J.inv_bs[a]), h = (int)(B.hi[a] * J.inv_bs[a]);
                blo[a] = max(0, min(l, J.nb[a] - 1));
                bhi[a] = max(blo[a], min(h, J.nb[a] - 1));
            } else {
                blo[a] = bhi[a] = 0;
            }
            olo[a] = 1;
            ohi[a] = 0;
        }
        int nbx = bhi[0] - blo[0] + 1, nby = bhi[1] - blo[1] + 1, nbz = bhi[2] - blo[2] + 1;
        int64_t sh_total = (int64_t)nbx * nby * nbz, sh_pos = 0;
        int ch_T = 0, ch_off = 0;
        bool ch_live = false;
        double UB = __builtin_inf();
        int nc = 0;
        bool lex = false, done = false;

        for (;;) {
            bool flush = false;
            // ======== gather ========
            while (!done && !flush) {
                if (!ch_live) {
                    if (sh_pos >= sh_total) {
                        // Shell finished: lower bound of every unvisited site.
                        bool complete = true;
                        double G = __builtin_inf();
                        for (int a = 0; a < DIM; ++a) {
                            const bool full = periodic ? (bhi[a] - blo[a] + 1 >= J.nb[a])
                                                       : (blo[a] == 0 && bhi[a] == J.nb[a] - 1);
                            if (full)
                                continue;
                            complete = false;
                            const double slack = J.L[a] * 0x1p-30;
                            if (periodic || blo[a] > 0)
                                G = fmin(G, B.lo[a] - ((double)blo[a] * J.bs[a] + slack));
                            if (periodic || bhi[a] < J.nb[a] - 1)
                                G = fmin(G, ((double)(bhi[a] + 1) * J.bs[a] - slack) - B.hi[a]);
                        }
                        if (complete) {
                            done = true;
                            break;
                        }
                        G = fmax(G, 0.0);
                        const double LB = (KIND == KV)   ? G * G
                                          : (KIND == KL) ? G * G - pmax
                                                         : pmin + G * rv;
                        if (LB > UB + M) {
                            done = true;
                            break;
                        }
                        for (int a = 0; a < DIM; ++a) {
                            olo[a] = blo[a];
                            ohi[a] = bhi[a];
                            if (periodic) {
                                if (bhi[a] - blo[a] + 1 < J.nb[a]) {
                                    blo[a] -= 1;
                                    bhi[a] += 1;
                                    if (bhi[a] - blo[a] + 1 > J.nb[a])
                                        bhi[a] = blo[a] + J.nb[a] - 1;
                                }
                            } else {
                                blo[a] = max(blo[a] - 1, 0);
                                bhi[a] = min(bhi[a] + 1, J.nb[a] - 1);
                            }
                        }
                        if (DIM == 2) {
                            olo[2] = ohi[2] = 0;
                        }
                        nbx = bhi[0] - blo[0] + 1;
                        nby = bhi[1] - blo[1] + 1;
                        nbz = bhi[2] - blo[2] + 1;
                        sh_total = (int64_t)nbx * nby * nbz;
                        sh_pos = 0;
                        continue;
                    }
                    // Next chunk of up to 64 bins of the box, skipping the old box.
                    const int64_t e = sh_pos + lane;
                    int cnt = 0, src = 0;
                    if (e < sh_total) {
                        const int ex = (int)(e % nbx);
                        const int64_t e2 = e / nbx;
                        const int ey = (int)(e2 % nby), ez = (int)(e2 / nby);
                        const int bx = blo[0] + ex, by = blo[1] + ey, bz = blo[2] + ez;
                        const bool old = bx >= olo[0] && bx <= ohi[0] && by >= olo[1] && by <= ohi[1] &&
                                         bz >= olo[2] && bz <= ohi[2];
                        if (!old) {
                            int wx = bx, wy = by, wz = bz;
                            if (periodic) {
                                wx = ((wx % J.nb[0]) + J.nb[0]) % J.nb[0];
                                wy = ((wy % J.nb[1]) + J.nb[1]) % J.nb[1];
                                wz = ((wz % J.nb[2]) + J.nb[2]) % J.nb[2];
                            }
                            const int lin = wx + J.nb[0] * (wy + J.nb[1] * wz);
                            src = J.bin_start[lin];
                            cnt = J.bin_start[lin + 1] - src;
                        }
                    }
                    const int inc = wave_inclusive_add(cnt, lane);
                    S.bcnt[lane] = inc;
                    S.bsrc[lane] = src;
                    ch_T = __shfl(inc, WAVE - 1);
                    ch_off = 0;
                    ch_live = ch_T > 0;
                    sh_pos += WAVE;
                    __syncthreads();
                    continue;
                }
                // Up to 64 sites of the chunk, one per lane.
                const int p = ch_off + lane;
                const bool valid = p < ch_T;
                double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
                int sid = 0, flags = 0;
                double lb = __builtin_inf(), ub = __builtin_inf(), dmn = 0.0, dmx = 0.0;
                if (valid) {
                    int lo = 0, hi = WAVE - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (S.bcnt[mid] > p)
                            hi = mid;
                        else
                            lo = mid + 1;
                    }
                    const int excl = lo == 0 ? 0 : S.bcnt[lo - 1];
                    const int pos = S.bsrc[lo] + (p - excl);
                    s = J.sites[pos];
                    sid = J.sidx[pos];
                    const double sc[3] = {s.x, s.y, s.z};
                    double qmin = 0.0, qmax = 0.0;
                    for (int a = 0; a < DIM; ++a) {
                        double sg = sc[a], dmin, dmax;
                        bool gen = false;
                        if (periodic) {
                            const int c1 = wrap_code(sc[a] - B.lo[a], J.H[a]);
                            const int c2 = wrap_code(sc[a] - B.hi[a], J.H[a]);
                            if (c1 == c2) {
                                flags |= c1 << (2 * a);
                                sg = sc[a] + code_off(c1, J.L[a]);
                            } else {
                                gen = true;
                            }
                        }
                        if (gen) {
                            flags |= FL_GENERIC;
                            dmin = 0.0;
                            dmax = J.H[a];
                        } else {
                            dmin = fmax(0.0, fmax(B.lo[a] - sg, sg - B.hi[a]));
                            dmax = fmax(fabs(sg - B.lo[a]), fabs(sg - B.hi[a]));
                        }
                        qmin += dmin * dmin;
                        qmax += dmax * dmax;
                    }
                    dmn = sqrt(qmin);
                    dmx = sqrt(qmax);
                    if (KIND == KV) {
                        lb = qmin;
                        ub = qmax;
                    } else if (KIND == KL) {
                        lb = qmin - s.w;
                        ub = qmax - s.w;
                    } else {
                        lb = s.w + dmn * rv;
                        ub = s.w + dmx * rv;
                    }
                }
                UB = fmin(UB, wave_min(ub));
                const bool keep = valid && lb <= UB + M;
                const unsigned long long km = __ballot(keep);
                if (keep) {
                    const int slot = nc + __popcll(km & lanes_below(lane));
                    S.cs[slot] = s;
                    S.cb[slot] = make_double2(lb, ub);
                    S.cq[slot] = make_double2(dmn, dmx);
                    S.cm[slot] = make_int2(sid, flags);
                }
                nc += __popcll(km);
                ch_off += WAVE;
                if (ch_off >= ch_T)
                    ch_live = false;
                __syncthreads();
                if (nc > CAP - WAVE) {
                    const double thr = UB + M;
                    nc = compact(S, nc, S.cb[lane].x <= thr, S.cb[lane + WAVE].x <= thr, lane);
                    if (nc > CAP - WAVE)
                        flush = true;
                }
            }

            // ======== prune, sort by index, evaluate ========
            if (nc > 0) {
                const double thr = UB + M;
                nc = compact(S, nc, S.cb[lane].x <= thr, S.cb[lane + WAVE].x <= thr, lane);
                if (nc > 1) {
                    const bool d0 = lane < nc && dominated<KIND, DIM>(S, nc, lane, J, B, M, sumL2_sqrt, rv);
                    const bool d1 = lane + WAVE < nc &&
                                    dominated<KIND, DIM>(S, nc, lane + WAVE, J, B, M, sumL2_sqrt, rv);
                    nc = compact(S, nc, !d0, !d1, lane);
                }
                // Rank by site index (indices are distinct), then permute in place.
                {
                    int r0 = 0, r1 = 0;
                    const int i0 = lane < nc ? S.cm[lane].x : 0;
                    const int i1 = lane + WAVE < nc ? S.cm[lane + WAVE].x : 0;
                    for (int t = 0; t < nc; ++t) {
                        const int it = S.cm[t].x;
                        r0 += it < i0;
                        r1 += it < i1;
                    }
                    double4 s0, s1;
                    int2 m0, m1;
                    if (lane < nc) {
                        s0 = S.cs[lane];
                        m0 = S.cm[lane];
                    }
                    if (lane + WAVE < nc) {
                        s1 = S.cs[lane + WAVE];
                        m1 = S.cm[lane + WAVE];
                    }
                    __syncthreads();
                    if (lane < nc) {
                        S.cs[r0] = s0;
                        S.cm[r0] = m0;
                    }
                    if (lane + WAVE < nc) {
                        S.cs[r1] = s1;
                        S.cm[r1] = m1;
                    }
                    __syncthreads();
                }
                // Exact keys, candidates in ascending index order.
                for (int k = 0; k < nc; ++k) {
                    const double4 s = S.cs[k];
                    const int2 m = S.cm[k];
                    const int idx = m.x, fl = m.y;
                    double c;
                    double dxv[RUN];
                    if (fl == 0) {
                        const double dy = s.y - yv;
                        if (DIM == 3) {
                            const double dz = s.z - zv;
                            c = dy * dy + dz * dz;
                        } else {
                            c = dy * dy;
                        }
#pragma unroll
                        for (int q = 0; q < RUN; ++q)
                            dxv[q] = s.x - xr[q];
                    } else if (!(fl & FL_GENERIC)) {
                        const double dy = (s.y - yv) + code_off((fl >> 2) & 3, J.L[1]);
                        if (DIM == 3) {
                            const double dz = (s.z - zv) + code_off((fl >> 4) & 3, J.L[2]);
                            c = dy * dy + dz * dz;
                        } else {
                            c = dy * dy;
                        }
                        const double ox = code_off(fl & 3, J.L[0]);
#pragma unroll
                        for (int q = 0; q < RUN; ++q)
                            dxv[q] = (s.x - xr[q]) + ox;
                    } else {
                        const double dy = periodic ? min_image(s.y - yv, J.H[1], J.L[1]) : s.y - yv;
                        if (DIM == 3) {
                            const double dz = periodic ? min_image(s.z - zv, J.H[2], J.L[2]) : s.z - zv;
                            c = dy * dy + dz * dz;
                        } else {
                            c = dy * dy;
                        }
#pragma unroll
                        for (int q = 0; q < RUN; ++q)
                            dxv[q] = periodic ? min_image(s.x - xr[q], J.H[0], J.L[0]) : s.x - xr[q];
                    }
                    if (!lex) {
#pragma unroll
                        for (int q = 0; q < RUN; ++q) {
                            const double key = dist_key<KIND>(dxv[q] * dxv[q] + c, s.w, v, rv);
                            const bool lt = key < best[q];
                            lab[q] = lt ? idx : lab[q];
                            best[q] = lt ? key : best[q];
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < RUN; ++q) {
                            const double key = dist_key<KIND>(dxv[q] * dxv[q] + c, s.w, v, rv);
                            const bool lt = key < best[q] || (key == best[q] && idx < lab[q]);
                            lab[q] = lt ? idx : lab[q];
                            best[q] = lt ? key : best[q];
                        }
                    }
                }
                lex = true;
                nc = 0;
                __syncthreads();
            }
            if (done)
                break;
        }
    }

    // ---- coalesced label stores (x fastest)
    if (mj < J.n[1] && mk < J.n[2]) {
        int32_t* out = J.labels + (int64_t)mi + (int64_t)J.n[0] * ((int64_t)mj + (int64_t)J.n[1] * mk);
        if (bad) {
#pragma unroll
            for (int q = 0; q < RUN; ++q)
                lab[q] = -1;
        }
        if (mi + RUN <= J.n[0] && ((uintptr_t)out & 15) == 0 && RUN % 4 == 0) {
#pragma unroll
            for (int q = 0; q < RUN; q += 4)
                *(int4*)(out + q) = make_int4(lab[q], lab[q + 1], lab[q + 2], lab[q + 3]);
        } else {
#pragma unroll
            for (int q = 0; q < RUN; ++q)
                if (mi + q < J.n[0])
                    out[q] = lab[q];
        }
    }
}

// Spreads consecutive tiles over one XCD: workgroups are dispatched to the
// eight XCDs round-robin, so workgroup b runs on XCD b % 8.  Give each XCD a
// contiguous range of tiles so that neighbouring tiles share its L2.
__device__ inline int64_t xcd_tile(int64_t b, int64_t G)
{
    const int64_t x = b & 7, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

template <int KIND, int DIM, int CFG>
__global__ __launch_bounds__(WAVE) void k_label_single(JobDev J)
{
    __shared__ WaveLds S;
    constexpr TileShape T = (DIM == 3) ? kShape3[CFG] : kShape2[CFG];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    label_tile<KIND, DIM, T.run, T.lx, T.ly, T.lz>(J, tile, S, threadIdx.x);
}

template <int KIND, int DIM>
__device__ void batch_tile(const JobDev& J, int64_t t, WaveLds& S, int lane)
{
    constexpr TileShape T = (DIM == 3) ? kShape3[0] : kShape2[0];
    label_tile<KIND, DIM, T.run, T.lx, T.ly, T.lz>(J, t, S, lane);
}

// Persistent batch kernel: the global tile enumeration (jobs one after the
// other) is cut into eight ranges, one per XCD; each wave takes tiles of its
// own XCD's range from an atomic counter and then helps the other ranges.
__global__ __launch_bounds__(WAVE) void k_label_batch(const JobDev* __restrict__ jobs, int njobs,
                                                      int64_t total, int32_t* counters)
{
    __shared__ WaveLds S;
    __shared__ int64_t got;
    const int lane = threadIdx.x;
    const int home = blockIdx.x & 7;
    for (int probe = 0; probe < 8; ++probe) {
        const int x = (home + probe) & 7;
        const int64_t rb = total * x / 8, re = total * (x + 1) / 8;
        for (;;) {
            if (lane == 0)
                got = rb + (int64_t)atomicAdd(&counters[x], 1);
            __syncthreads();
            const int64_t g = got;
            __syncthreads();
            if (g >= re)
                break;
            // job of tile g: largest j with tile_begin <= g
            int lo = 0, hi = njobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].tile_begin <= g)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const int j = __builtin_amdgcn_readfirstlane(lo);
            const JobDev& J = jobs[j];
            const int64_t t = g - J.tile_begin;
            const int code = J.kind == KIND_VORONOI ? KV
                             : J.kind == KIND_LAGUERRE ? KL
                             : (J.jm_div ? KJD : KJM);
            if (J.ndim == 3) {
                switch (code) {
                case KV: batch_tile<KV, 3>(J, t, S, lane); break;
                case KL: batch_tile<KL, 3>(J, t, S, lane); break;
                case KJM: batch_tile<KJM, 3>(J, t, S, lane); break;
                default: batch_tile<KJD, 3>(J, t, S, lane); break;
                }
            } else {
                switch (code) {
                case KV: batch_tile<KV, 2>(J, t, S, lane); break;
                case KL: batch_tile<KL, 2>(J, t, S, lane); break;
                case KJM: batch_tile<KJM, 2>(J, t, S, lane); break;
                default: batch_tile<KJD, 2>(J, t, S, lane); break;
                }
            }
            __syncthreads();
        }
    }
}

template <int KIND, int DIM>
hipError_t launch_single_cfg(const JobDev& job, hipStream_t s)
{
    const unsigned grid = (unsigned)job.ntiles;
    switch (job.cfg) {
    case 0: k_label_single<KIND, DIM, 0><<<grid, WAVE, 0, s>>>(job); break;
    case 1: k_label_single<KIND, DIM, 1><<<grid, WAVE, 0, s>>>(job); break;
    default: k_label_single<KIND, DIM, 2><<<grid, WAVE, 0, s>>>(job); break;
    }
    return hipGetLastError();
}

template <int DIM>
hipError_t launch_single_dim(const JobDev& job, hipStream_t s)
{
    if (job.kind == KIND_VORONOI)
        return launch_single_cfg<KV, DIM>(job, s);
    if (job.kind == KIND_LAGUERRE)
        return launch_single_cfg<KL, DIM>(job, s);
    if (job.jm_div)
        return launch_single_cfg<KJD, DIM>(job, s);
    return launch_single_cfg<KJM, DIM>(job, s);
}

}  // namespace

hipError_t launch_label_single(const JobDev& job, hipStream_t s)
{
    if (job.ntiles <= 0 || job.ntiles > 0x7fffffffLL)
        return hipErrorInvalidValue;
    return job.ndim == 3 ? launch_single_dim<3>(job, s) : launch_single_dim<2>(job, s);
}

int label_batch_grid(int device)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    return cus * 16;
}

hipError_t launch_label_batch(const JobDev* jobs_dev, int njobs, int ndim_mask, int64_t total_tiles,
                              int32_t* counters, int grid, hipStream_t s)
{
    (void)ndim_mask;
    if (total_tiles <= 0)
        return hipSuccess;
    k_label_batch<<<grid, WAVE, 0, s>>>(jobs_dev, njobs, total_tiles, counters);
    return hipGetLastError();
}

}  // namespace vt
