// HIP kernels of the semantic TSDF integrator (gfx950, wave64).
//
// One frame runs as five kernels on the map's stream:
//   1. ray_walk_emit  one lane per point: pose application, ray, band, voxel
//                     walk (Sec. III-A), truncation gate.  The leaves the
//                     block's rays touch are collected in an LDS table, so each
//                     (block, leaf) makes one staging insert and one bucket
//                     reservation; every kept (voxel, point) observation is
//                     written as a pair.
//   2. leaf_plan      one lane per touched leaf: find it in the map (or number
//                     it as new), number record pages for newly touched 8x8
//                     slabs, allocate its pair bucket.
//   3. pair_bucket    one lane per pair: scatter into its leaf's bucket.
//   4. leaf_acc       geometry and int32 labels (K <= 32): one workgroup per
//                     touched leaf (or one wave per small leaf) adds every pair
//                     into its voxel's LDS accumulators with integer atomics --
//                     observation counts, class counts, fixed-point distance
//                     sums -- and one lane per touched voxel applies them, Eq.
//                     (1)-(2) for D and W and Eq. (6) for the class counts.
//      leaf_fuse      probability or logit rows, the open set, the most-recent
//                     modes: counting sort of the bucket by voxel offset in LDS,
//                     then by point index inside each voxel, and the combine of
//                     every touched voxel in point order (the open set's Eqs.
//                     (11)-(14) with lambda = 2 nu = W in k_voxel_combine).
//   5. frame_commit   one workgroup: counters, status, frame reset.
// Kernels 1-3 only read the map, and kernel 4 writes it only if the frame's new
// leaves and record pages fit (decided from totals that kernel 2 completed), so
// a frame that does not fit changes nothing.  No floating-point atomics are
// used: integer sums are exact in any order and every floating-point sum runs
// in point order, so results are bitwise repeatable and independent of launch
// shapes.
//
// The geometric decision path (pose, ray, walk, gate) is a fixed sequence of
// binary32 operations; build with -ffp-contract=off so that only the fmaf()
// calls written here fuse, and with correctly rounded division and sqrt.

#include <hip/hip_runtime.h>

#include <mutex>

#include "slim_internal.h"
#include "slimvdb.h"

namespace slim {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t leaf_hash(unsigned long long k, uint32_t mask)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (uint32_t)k & mask;
}

// Slot of a leaf in the map's table, or -1.
__device__ int32_t map_find(const MapDev &md, unsigned long long key)
{
    uint32_t h = leaf_hash(key, md.hmask);
    for (uint32_t probe = 0; probe <= md.hmask; ++probe) {
        const uint4 e = *(const uint4 *)&md.htab[h];
        const unsigned long long k = ((unsigned long long)e.y << 32) | e.x;
        if (k == key) return (int32_t)e.z;
        if (k == kEmptyKey) return -1;
        h = (h + 1) & md.hmask;
    }
    return -1;
}

// Inserts a leaf known to be absent, in two steps so that the first probe's
// round trip can overlap other loads: map_insert_start claims the leaf's home
// slot if it is free (one compare-and-swap) and map_insert_finish, given that
// result, probes on if it was taken and stores the slot.  The table is at
// most half full.
__device__ __forceinline__ unsigned long long map_insert_start(const MapDev &md, unsigned long long key,
                                                               uint32_t *h)
{
    *h = leaf_hash(key, md.hmask);
    return atomicCAS(&md.htab[*h].key, kEmptyKey, key);
}

__device__ void map_insert_finish(const MapDev &md, unsigned long long key, int32_t slot, uint32_t h,
                                  unsigned long long prev)
{
    for (uint32_t probe = 0; probe <= md.hmask; ++probe) {
        if (prev == kEmptyKey) {
            md.htab[h].val = slot;
            return;
        }
        h = (h + 1) & md.hmask;
        prev = atomicCAS(&md.htab[h].key, kEmptyKey, key);
    }
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// ---------------------------------------------------------------------------
// geometry (binary32, fixed operation order)
// ---------------------------------------------------------------------------

struct Ray {
    float p[3];   // point relative to the anchor corner
    float u[3];   // unit direction
    float t0, t1; // band
};

__device__ __forceinline__ bool make_ray(const FrameParams &fp, float x, float y, float z, Ray &ry)
{
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) return false;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        ry.p[a] = fmaf(fp.R[3 * a + 0], x, fmaf(fp.R[3 * a + 1], y, fmaf(fp.R[3 * a + 2], z, fp.t[a])));
    const float d0 = ry.p[0] - fp.t[0], d1 = ry.p[1] - fp.t[1], d2 = ry.p[2] - fp.t[2];
    const float r = sqrtf(fmaf(d2, d2, fmaf(d1, d1, d0 * d0)));
    if (!(r > 0.0f) || !isfinite(r) || r < fp.rmin || r > fp.rmax) return false;
    ry.u[0] = d0 / r;
    ry.u[1] = d1 / r;
    ry.u[2] = d2 / r;
    ry.t0 = fmaxf(r - fp.tau, 0.0f);
    ry.t1 = r + fp.tau;
    return true;
}

// Sensor-frame point i: given directly, as range * unit direction (one
// binary32 product per component), or back-projected from pixel i of a depth
// image, ((u - cx) / fx) d, ((v - cy) / fy) d, d, rounded in that order (a
// depth that is not finite and positive gives a rejected point).
__device__ __forceinline__ void load_point(const FrameParams &fp, int i, float &x, float &y, float &z)
{
    if (fp.pts) {
        x = fp.pts[3 * i + 0];
        y = fp.pts[3 * i + 1];
        z = fp.pts[3 * i + 2];
    } else if (fp.depth) {
        const int v = i / fp.width, u = i - v * fp.width;
        const float d = fp.depth[i];
        if (!(d > 0.0f) || !isfinite(d)) {
            x = y = z = NAN;
            return;
        }
        x = (((float)u - fp.cx) / fp.fx) * d;
        y = (((float)v - fp.cy) / fp.fy) * d;
        z = d;
    } else {
        const float r = fp.ranges[i];
        x = r * fp.dirs[3 * i + 0];
        y = r * fp.dirs[3 * i + 1];
        z = r * fp.dirs[3 * i + 2];
    }
}

// Amanatides-Woo walk over the band of the ray from the sensor origin
// (fp.t).  Calls visit(cx, cy, cz) per cell (anchor-relative).  Ties between
// axes step the lowest axis first, one axis per step; the walk stops when the
// next boundary lies beyond t1, or after maxsteps cells.
// Start of the walk: first cell c, step direction, first boundary crossing
// tm and crossing interval td per axis (tm = td = inf on an axis the ray does
// not move along).
struct WalkState {
    int c[3], stp[3];
    float tm[3], td[3];
};

// Returns false when a start cell lies 2^30 or more cells from the anchor: its
// key is then outside |k| < 2^20 whatever the anchor, so the point is rejected
// (and the cell index never overflows an int while the walk steps on).
constexpr float kCellLimit = 1073741824.0f;  // 2^30

__device__ __forceinline__ bool walk_start(const FrameParams &fp, const Ray &ry, WalkState &w)
{
    const float vs = fp.vs, t0 = ry.t0;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float s = fmaf(t0, ry.u[a], fp.t[a]);
        const float fc = floorf(s / vs);
        ok = ok && fabsf(fc) < kCellLimit;
        w.c[a] = fabsf(fc) < kCellLimit ? (int)fc : 0;
        if (ry.u[a] > 0.0f) {
            w.stp[a] = 1;
            w.tm[a] = t0 + fmaf((float)(w.c[a] + 1), vs, -s) / ry.u[a];
            w.td[a] = vs / ry.u[a];
        } else if (ry.u[a] < 0.0f) {
            w.stp[a] = -1;
            w.tm[a] = t0 + fmaf((float)w.c[a], vs, -s) / ry.u[a];
            w.td[a] = -vs / ry.u[a];
        } else {
            w.stp[a] = 0;
            w.tm[a] = INFINITY;
            w.td[a] = INFINITY;
        }
    }
    return ok;
}

// Axis of the next step (ties step the lowest axis) and the ray parameter of
// the boundary it crosses.
__device__ __forceinline__ int walk_axis(const WalkState &w, float &tnext)
{
    const bool xy = w.tm[0] <= w.tm[1];
    const int ax = xy ? (w.tm[0] <= w.tm[2] ? 0 : 2) : (w.tm[1] <= w.tm[2] ? 1 : 2);
    tnext = ax == 0 ? w.tm[0] : (ax == 1 ? w.tm[1] : w.tm[2]);
    return ax;
}

// One step along axis ax, written as selects (no branch per axis).
__device__ __forceinline__ void walk_step(WalkState &w, int ax)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool on = ax == a;
        w.c[a] += on ? w.stp[a] : 0;
        const float nt = w.tm[a] + w.td[a];
        w.tm[a] = on ? nt : w.tm[a];
    }
}

// Amanatides-Woo walk over the band of the ray from the sensor origin
// (fp.t).  Calls visit(cx, cy, cz) per cell (anchor-relative).  Ties between
// axes step the lowest axis first, one axis per step; the walk stops when the
// next boundary lies beyond t1, or after maxsteps cells.
template <class Visit>
__device__ __forceinline__ bool band_walk(const FrameParams &fp, const Ray &ry, Visit &&visit)
{
    WalkState w;
    if (!walk_start(fp, ry, w)) return false;
    for (int it = 0; it < fp.maxsteps; ++it) {
        visit(w.c[0], w.c[1], w.c[2]);
        float tnext;
        const int ax = walk_axis(w, tnext);
        if (tnext > ry.t1) break;
        walk_step(w, ax);
    }
    return true;
}

// Signed distance (binary32) of a cell centre to the point along the ray;
// positive in front of the surface.
__device__ __forceinline__ float cell_sdf(const FrameParams &fp, const Ray &ry, int cx, int cy, int cz)
{
    const float h = 0.5f * fp.vs;
    const float qx = fmaf(-(float)cx, fp.vs, ry.p[0]) - h;
    const float qy = fmaf(-(float)cy, fp.vs, ry.p[1]) - h;
    const float qz = fmaf(-(float)cz, fp.vs, ry.p[2]) - h;
    return fmaf(qz, ry.u[2], fmaf(qy, ry.u[1], qx * ry.u[0]));
}

__device__ __forceinline__ bool key_ok(int k) { return k > -kKeyLimit && k < kKeyLimit; }

// ---------------------------------------------------------------------------
// block-wide helpers (blockDim.x a multiple of 64, at most 256)
// ---------------------------------------------------------------------------

// Exclusive prefix sum over the block of one value per thread; *total gets
// the block sum.  Uses wsum[4] of LDS.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t *total)
{
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    const int nw = (int)(blockDim.x >> 6);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < w) before += wsum[q];
        if (q < nw) tot += wsum[q];
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

// Exclusive prefix sum of 512 LDS counters by 256 threads.
__device__ void block_scan512(const uint32_t *in, uint32_t *out, uint32_t *wsum)
{
    const int t = threadIdx.x;
    const uint32_t a = in[2 * t], b = in[2 * t + 1];
    uint32_t total;
    const uint32_t ex = block_excl_scan(a + b, wsum, &total);
    out[2 * t] = ex;
    out[2 * t + 1] = ex + a;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// 1. ray walk and pair emission
// ---------------------------------------------------------------------------

constexpr int kWaveItemPairs = 256;  // leaves with at most this many pairs are one wave's work
constexpr int kMaxRuns = 8;  // leaf runs per ray; sdf_trunc <= 6 voxel_size keeps a ray within this
static_assert(kWalkTable >= kWalkThreads * kMaxRuns, "the walk table must hold every run of a block");

__device__ __forceinline__ uint32_t lds_hash(unsigned long long k)
{
    return (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> 40) & (kWalkTable - 1);
}

// Staging-table position of a leaf for the walk: one compare-and-swap per
// probe (an empty slot is claimed, a slot holding the key is found), so the
// common case is one round trip.  *fresh is true for the claiming caller.
__device__ __forceinline__ uint32_t stage_leaf_cas(const MapDev &md, unsigned long long key, bool *fresh)
{
    *fresh = false;
    uint32_t h = leaf_hash(key, md.hmask);
    for (uint32_t probe = 0; probe <= md.hmask; ++probe) {
        const unsigned long long prev = atomicCAS(&md.skeys[h], kEmptyKey, key);
        if (prev == kEmptyKey) {
            *fresh = true;
            return h;
        }
        if (prev == key) return h;
        h = (h + 1) & md.hmask;
    }
    return kNoPos;
}

// Block-local table of the leaves a walk block's rays touch.
// Kept small enough for three workgroups per CU: slab masks are 8-bit fields,
// four to a word, and entry lists 16-bit.
static_assert(kWalkTable <= 65536, "walk-table entries are listed as 16-bit indices");
struct WalkShared {
    unsigned long long t_key[kWalkTable];
    uint32_t t_cnt[kWalkTable];       // pairs of this block in the leaf, then their first bucket rank
    uint32_t t_pos[kWalkTable];       // staging position
    uint32_t t_slab[kWalkTable / 4];  // x-slabs of the leaf this block touches (8 bits per entry)
    uint16_t t_list[kWalkTable];      // occupied entries
    uint16_t t_fresh[kWalkTable];     // entries whose staging insert this block made
    uint32_t s_n, s_nfresh, s_pair_base, wsum[4];
};

// One block of the walk: rays blk * blockDim.x + [0, blockDim.x) of a frame.
__device__ __forceinline__ void walk_emit_block(const FrameParams &fp, const MapDev &md, int blk, WalkShared &ws)
{
    unsigned long long *t_key = ws.t_key;
    uint32_t *t_cnt = ws.t_cnt, *t_pos = ws.t_pos, *t_slab = ws.t_slab;
    uint16_t *t_list = ws.t_list, *t_fresh = ws.t_fresh;
    uint32_t &s_n = ws.s_n, &s_nfresh = ws.s_nfresh, &s_pair_base = ws.s_pair_base;
    uint32_t *wsum = ws.wsum;

    const int tid = threadIdx.x;
    const int i = blk * blockDim.x + tid;
    // the point is loaded first: its latency overlaps the table clear
    Ray ry;
    bool valid = false;
    if (i < fp.n) {
        float x, y, z;
        load_point(fp, i, x, y, z);
        valid = make_ray(fp, x, y, z, ry);
        if (valid && fp.sem_kind == SLIM_IN_LABEL_I32) {
            const int lab = ((const int32_t *)fp.sem)[i];
            valid = lab >= 0 && lab < fp.K;
        }
    }
    for (int e = tid; e < kWalkTable; e += blockDim.x) {
        t_key[e] = kEmptyKey;
        t_cnt[e] = 0;
    }
    for (int e = tid; e < kWalkTable / 4; e += blockDim.x) t_slab[e] = 0;
    if (tid == 0) {
        s_n = 0;
        s_nfresh = 0;
    }
    __syncthreads();

    // pass 1: count kept cells, check the key range, record the leaf runs.
    // The current run is accumulated in clen/cslab; the run arrays are
    // written only when a run ends.  The walk is recorded for pass 2: the
    // first cell, the axis of every step (2 bits each) and which cells passed
    // the gate.
    uint32_t cnt = 0;
    int nruns = 0;
    unsigned long long rkey[kMaxRuns];
    uint32_t rlen[kMaxRuns], rslab[kMaxRuns];
#pragma unroll
    for (int q = 0; q < kMaxRuns; ++q) {
        rkey[q] = kEmptyKey;
        rlen[q] = 0;
        rslab[q] = 0;
    }
    int c0[3] = {0, 0, 0};
    int nvis = 0;
    unsigned long long steps[2] = {0ull, 0ull}, kept = 0ull;
    if (valid) {
        unsigned long long cur = kEmptyKey;
        uint32_t clen = 0, cslab = 0;
        WalkState w;
        bool inrange = walk_start(fp, ry, w);
        c0[0] = w.c[0];
        c0[1] = w.c[1];
        c0[2] = w.c[2];
        for (int it = 0; it < (inrange ? fp.maxsteps : 0); ++it) {
            const int kx = fp.a[0] + w.c[0], ky = fp.a[1] + w.c[1], kz = fp.a[2] + w.c[2];
            if (!(key_ok(kx) && key_ok(ky) && key_ok(kz))) {
                inrange = false;
                break;
            }
            nvis = it + 1;
            if (cell_sdf(fp, ry, w.c[0], w.c[1], w.c[2]) > -fp.tau) {
                kept |= 1ull << it;
                const unsigned long long lk = pack_leaf(kx >> 3, ky >> 3, kz >> 3);
                if (lk != cur) {
#pragma unroll
                    for (int q = 0; q < kMaxRuns; ++q) {
                        if (q == nruns - 1) {
                            rlen[q] = clen;
                            rslab[q] = cslab;
                        }
                        if (q == nruns) rkey[q] = lk;
                    }
                    cur = lk;
                    nruns++;
                    clen = 0;
                    cslab = 0;
                }
                clen++;
                cslab |= 1u << (kx & 7);
                cnt++;
            }
            float tnext;
            const int ax = walk_axis(w, tnext);
            if (tnext > ry.t1) break;
            steps[it >> 5] |= (unsigned long long)ax << (2 * (it & 31));
            walk_step(w, ax);
        }
#pragma unroll
        for (int q = 0; q < kMaxRuns; ++q)
            if (q == nruns - 1) {
                rlen[q] = clen;
                rslab[q] = cslab;
            }
        if (!inrange || nruns > kMaxRuns) valid = false;
    }
    if (!valid) {
        cnt = 0;
        nruns = 0;
    }

    // runs into the block table: local rank of each run inside its leaf
    uint32_t rent[kMaxRuns], rloc[kMaxRuns];
#pragma unroll
    for (int q = 0; q < kMaxRuns; ++q) {
        rent[q] = kWalkTable;
        rloc[q] = 0;
        if (q < nruns) {
            // distinct keys <= runs of the block <= table size, so a free or
            // matching entry always exists; the probe bound is a safeguard
            const unsigned long long key = rkey[q];
            uint32_t h = lds_hash(key);
            bool found = false;
            for (int probe = 0; probe < kWalkTable && !found; ++probe) {
                unsigned long long k = t_key[h];
                if (k == kEmptyKey) {
                    k = atomicCAS(&t_key[h], kEmptyKey, key);
                    if (k == kEmptyKey) {
                        t_list[atomicAdd(&s_n, 1u)] = (uint16_t)h;
                        k = key;
                    }
                }
                if (k == key) found = true;
                else h = (h + 1) & (kWalkTable - 1);
            }
            if (found) {
                rent[q] = h;
                rloc[q] = atomicAdd(&t_cnt[h], rlen[q]);
                atomicOr(&t_slab[h >> 2], rslab[q] << (8u * (h & 3u)));
            } else {
                atomicOr(&md.fs->frame_err.v, 1u);  // pairs of this run are dropped, frame rejected
            }
        }
    }
    const uint32_t rejected_block = __syncthreads_count((i < fp.n) && !valid);

    // the block's pair range is reserved while the leaves are staged
    uint32_t total;
    const uint32_t off = block_excl_scan(cnt, wsum, &total);
    uint32_t pair_base = 0;
    if (tid == 0) {
        if (total) pair_base = atomicAdd(&md.fs->pairs.v, total);
        if (rejected_block) atomicAdd(&md.fs->rejected.v, rejected_block);
    }
    // one staging lookup, one bucket reservation and one slab update per leaf of the block
    const uint32_t nloc = s_n;
    for (uint32_t e = tid; e < nloc; e += blockDim.x) {
        const uint32_t h = t_list[e];
        bool fresh;
        const uint32_t pos = stage_leaf_cas(md, t_key[h], &fresh);
        t_pos[h] = pos;
        if (pos != kNoPos) {
            t_cnt[h] = atomicAdd(&md.pos_count[pos], t_cnt[h]);
            atomicOr(&md.pos_slab[pos], (t_slab[h >> 2] >> (8u * (h & 3u))) & 0xFFu);
            if (fresh) t_fresh[atomicAdd(&s_nfresh, 1u)] = (uint16_t)h;
        } else {
            atomicOr(&md.fs->frame_err.v, 1u);
        }
    }
    if (tid == 0) s_pair_base = pair_base;
    __syncthreads();
    // wave 0 reserves the block's touched-list range now and writes it after
    // its own pairs, so the reservation's latency overlaps pass 2
    const uint32_t nfresh = s_nfresh;
    uint32_t fresh_base = 0;
    if (tid == 0 && nfresh) fresh_base = atomicAdd(&md.fs->n_touched.v, nfresh);

    // pass 2: write the pairs, replaying the recorded walk
    const uint32_t o = s_pair_base + off;
    const bool fits = o + cnt <= md.pair_cap;
    uint32_t j = 0;
    int run = -1;
    unsigned long long cur = kEmptyKey;
    uint32_t pos = kNoPos, rank = 0;
    const int stp[3] = {ry.u[0] > 0.0f ? 1 : -1, ry.u[1] > 0.0f ? 1 : -1, ry.u[2] > 0.0f ? 1 : -1};
    int cc[3] = {c0[0], c0[1], c0[2]};
    if (cnt == 0) nvis = 0;
    for (int vi = 0; vi < nvis; ++vi) {
        if (vi > 0) {
            const int si = vi - 1;
            const int ax = (int)((steps[si >> 5] >> (2 * (si & 31))) & 3ull);
#pragma unroll
            for (int a = 0; a < 3; ++a) cc[a] += ax == a ? stp[a] : 0;
        }
        if (!((kept >> vi) & 1ull)) continue;
        const int cx = cc[0], cy = cc[1], cz = cc[2];
        const float s = cell_sdf(fp, ry, cx, cy, cz);
        const int kx = fp.a[0] + cx, ky = fp.a[1] + cy, kz = fp.a[2] + cz;
        const unsigned long long lk = pack_leaf(kx >> 3, ky >> 3, kz >> 3);
        if (lk != cur) {
            cur = lk;
            run++;
#pragma unroll
            for (int q = 0; q < kMaxRuns; ++q)
                if (q == run) {
                    pos = rent[q] < (uint32_t)kWalkTable ? t_pos[rent[q]] : kNoPos;
                    rank = rent[q] < (uint32_t)kWalkTable ? t_cnt[rent[q]] + rloc[q] : 0u;
                }
        }
        const uint32_t voff = (uint32_t)(((kx & 7) << 6) | ((ky & 7) << 3) | (kz & 7));
        if (fits || o + j < md.pair_cap) {
            md.pairs[o + j] = make_uint4(pos, rank++, (voff << kPidBits) | (fp.pid_base + (uint32_t)i),
                                         __float_as_uint(fminf(s, fp.tau)));
        }
        j++;
    }
    if (tid < 64 && nfresh) {
        const uint32_t base = __shfl(fresh_base, 0, 64);
        for (uint32_t e = tid; e < nfresh; e += 64) {
            const uint32_t h = t_fresh[e];
            md.touched[base + e] = t_pos[h];
            md.touched_key[base + e] = t_key[h];
        }
    }
}

__global__ __launch_bounds__(kWalkThreads) void k_ray_walk_emit(FrameParams fp, MapDev md)
{
    __shared__ WalkShared ws;
    walk_emit_block(fp, md, blockIdx.x, ws);
}

// Map of a block of a batched launch (frame of a multi-frame pass): the last i
// with start[i] <= blk.
__device__ __forceinline__ int batch_map(const int *start, int nmaps, int blk)
{
    int lo = 0, hi = nmaps;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= blk) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kWalkThreads) void k_ray_walk_emit_batch(MapBatch mb)
{
    __shared__ WalkShared ws;
    const int i = batch_map(mb.walk_start, mb.nmaps, blockIdx.x);
    walk_emit_block(mb.fps[i], mb.mds[i], blockIdx.x - mb.walk_start[i], ws);
}

// The rays of every frame of a multi-frame pass into one staging buffer.
__global__ __launch_bounds__(kWalkThreads) void k_ray_walk_emit_pass(PassWalk pw, MapDev md)
{
    __shared__ WalkShared ws;
    const int f = batch_map(pw.blk_start, pw.nframes, blockIdx.x);
    walk_emit_block(pw.fp[f], md, blockIdx.x - pw.blk_start[f], ws);
}

// Frame (within a multi-frame pass) of sort-key point index p.
__device__ __forceinline__ int pass_frame(const FrameParams &fp, uint32_t p)
{
    int f = 0;
#pragma unroll
    for (int q = 1; q < kPassFrames; ++q) f += (q < fp.nsub && p >= fp.sub_start[q]) ? 1 : 0;
    return f;
}

// Class label of the observation with sort-key point index p.
__device__ __forceinline__ int32_t point_label(const FrameParams &fp, uint32_t p)
{
    if (fp.nsub <= 1) return ((const int32_t *)fp.sem)[p];
    const int f = pass_frame(fp, p);
    return ((const int32_t *)fp.sub_sem[f])[p - fp.sub_start[f]];
}

// ---------------------------------------------------------------------------
// 2. leaf planning
// ---------------------------------------------------------------------------

__device__ __forceinline__ void leaf_plan_range(const FrameParams &fp, const MapDev &md, uint32_t blk, uint32_t nblk)
{
    // work lists: the sorting leaf kernel splits a leaf with more pairs than
    // LDS holds into x-slab items and gives a wave leaves of up to
    // kWaveItemPairs pairs; the accumulating one takes every leaf whole
    const bool acc = accum_path(fp);
    const uint32_t slab_cap = (uint32_t)kLeafLdsPairs, wave_cap = acc ? (uint32_t)kAccWavePairs : (uint32_t)kWaveItemPairs;
    const uint32_t big_lim = acc ? 0xFFFFFFFFu : (md.slab_pairs > 0 ? min((uint32_t)md.slab_pairs, slab_cap) : slab_cap);
    const uint32_t small_lim = md.wave_pairs > 0 ? min((uint32_t)md.wave_pairs, wave_cap) : wave_cap;
    const uint32_t nt = md.fs->n_touched.v;
    const unsigned long long pused = md.st->pages_used;
    const uint32_t stride = nblk * blockDim.x;
    for (uint32_t jb = blk * blockDim.x; jb < nt; jb += stride) {
        const uint32_t j = jb + threadIdx.x;
        const bool act = j < nt;
        int32_t slot = -1;
        uint32_t npairs = 0, pos = 0, need = 0;
        unsigned long long key = kEmptyKey;
        uint4 occ[4] = {make_uint4(0u, 0u, 0u, 0u), make_uint4(0u, 0u, 0u, 0u), make_uint4(0u, 0u, 0u, 0u),
                        make_uint4(0u, 0u, 0u, 0u)};
        int pg[kLeafPages];
#pragma unroll
        for (int q = 0; q < kLeafPages; ++q) pg[q] = -1;
        if (act) {
            pos = md.touched[j];
            key = md.touched_key[j];
            slot = map_find(md, key);
            npairs = md.pos_count[pos];
            uint32_t have = 0;
            if (slot >= 0) {
                const int4 p0 = ((const int4 *)md.leaf_page)[2 * slot], p1 = ((const int4 *)md.leaf_page)[2 * slot + 1];
                pg[0] = p0.x; pg[1] = p0.y; pg[2] = p0.z; pg[3] = p0.w;
                pg[4] = p1.x; pg[5] = p1.y; pg[6] = p1.z; pg[7] = p1.w;
#pragma unroll
                for (int q = 0; q < 4; ++q) occ[q] = ((const uint4 *)md.leaf_occ)[(size_t)slot * 4 + q];
#pragma unroll
                for (int q = 0; q < kLeafPages; ++q) have |= (pg[q] >= 0 ? 1u : 0u) << q;
            }
            need = md.pos_slab[pos] & ~have & 0xFFu;
        }
        // a leaf with more pairs than the leaf kernel holds in LDS becomes one
        // work item per touched x-slab
        const uint32_t tslabs = act ? md.pos_slab[pos] & 0xFFu : 0u;
        const bool big = act && npairs > big_lim;
        // the other leaves: one workgroup each, or one wave each if small
        const bool small = act && npairs <= small_lim;
        const bool med = act && !big && !small;
        // the larger workgroup and wave leaves are listed from the front of
        // their arrays, the smaller ones from the back
        const bool medf = med && npairs > min(big_lim, slab_cap) / 2, medb = med && !medf;
        const bool smallf = small && npairs > small_lim / 4, smallb = small && !smallf;
        // eight reservations with six atomics in flight together (two list
        // counters share each 64-bit word)
        const uint32_t want[4] = {(act && slot < 0) ? 1u : 0u, (uint32_t)__popc(need), npairs,
                                  big ? (uint32_t)__popc(tslabs) : 0u};
        uint32_t incl[4], total[4], base[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            incl[q] = wave_incl_scan(want[q]);
            total[q] = __shfl(incl[q], 63, 64);
        }
        const uint32_t mincl = wave_incl_scan(medf ? 1u : 0u), sincl = wave_incl_scan(smallf ? 1u : 0u);
        const uint32_t mincb = wave_incl_scan(medb ? 1u : 0u), sincb = wave_incl_scan(smallb ? 1u : 0u);
        const unsigned long long lt = ((unsigned long long)__shfl(sincl, 63, 64) << 32) | __shfl(mincl, 63, 64);
        const unsigned long long ltb = ((unsigned long long)__shfl(sincb, 63, 64) << 32) | __shfl(mincb, 63, 64);
        unsigned long long lbase = 0, lbaseb = 0;
        if (lane_id() == 63) {
            if (total[0]) base[0] = atomicAdd(&md.fs->new_leaves.v, total[0]);
            if (total[1]) base[1] = atomicAdd(&md.fs->new_pages.v, total[1]);
            if (total[2]) base[2] = atomicAdd(&md.fs->pair_cursor.v, total[2]);
            if (total[3]) base[3] = atomicAdd(&md.fs->work_big.v, total[3]);
            if (lt) lbase = atomicAdd((unsigned long long *)&md.fs->n_lists, lt);
            if (ltb) lbaseb = atomicAdd((unsigned long long *)&md.fs->n_lists_tail, ltb);
        }
        uint32_t got[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) got[q] = __shfl(base[q], 63, 64) + incl[q] - want[q];
        const unsigned long long lb = __shfl(lbase, 63, 64), lbb = __shfl(lbaseb, 63, 64);
        const uint32_t newleaf = got[0], pbase = got[1], bstart = got[2], ibase = got[3];
        const uint32_t last = md.hmask;  // the item arrays of the lists hold hmask + 1 entries
        LeafItem *dst = nullptr;
        if (medf) dst = &md.items[(uint32_t)lb + mincl - 1u];
        if (smallf) dst = &md.items_small[(uint32_t)(lb >> 32) + sincl - 1u];
        if (medb) dst = &md.items[last - ((uint32_t)lbb + mincb - 1u)];
        if (smallb) dst = &md.items_small[last - ((uint32_t)(lbb >> 32) + sincb - 1u)];
        if (big) {
            // the leaf's slab items sit at ibase .. ibase + slabs - 1, its item at
            // ibase; every work entry below work_cap is written, so the leaf
            // kernel never reads an unwritten one (a frame that overflows the
            // work list is not applied)
            if (ibase < md.work_cap) dst = &md.items_big[ibase];
            uint32_t r = 0;
            for (int q = 0; q < kLeafPages; ++q)
                if ((tslabs >> q) & 1u) {
                    if (ibase + r < md.work_cap) md.work[ibase + r] = make_int2((int)ibase, q);
                    else atomicOr(&md.fs->frame_err.v, 1u);
                    r++;
                }
        }
        if (act) {
            uint32_t r = 0;
#pragma unroll
            for (int q = 0; q < kLeafPages; ++q)
                if ((need >> q) & 1u) pg[q] = (int)(pused + pbase + r++);
            md.pos_pages[2 * pos] = make_int4(pg[0], pg[1], pg[2], pg[3]);
            md.pos_pages[2 * pos + 1] = make_int4(pg[4], pg[5], pg[6], pg[7]);
            md.pos_plan[pos] = make_int4(slot, slot < 0 ? (int)newleaf : -1, (int)bstart, 0);
        }
        if (dst) {
            // the leaf kernel's item: header, pages, occupancy before this frame
            uint4 *it = (uint4 *)dst;
            it[0] = make_uint4(pos, npairs, bstart, (uint32_t)(slot >= 0 ? slot : -1 - (int)newleaf));
            it[1] = make_uint4(tslabs, 0u, (uint32_t)key, (uint32_t)(key >> 32));
            it[2] = make_uint4((uint32_t)pg[0], (uint32_t)pg[1], (uint32_t)pg[2], (uint32_t)pg[3]);
            it[3] = make_uint4((uint32_t)pg[4], (uint32_t)pg[5], (uint32_t)pg[6], (uint32_t)pg[7]);
#pragma unroll
            for (int q = 0; q < 4; ++q) it[4 + q] = occ[q];
        }
    }
}

__global__ __launch_bounds__(256) void k_leaf_plan(FrameParams fp, MapDev md)
{
    leaf_plan_range(fp, md, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_leaf_plan_batch(MapBatch mb)
{
    const int i = batch_map(mb.plan_first, mb.nmaps, blockIdx.x);
    leaf_plan_range(mb.fps[i], mb.mds[i], blockIdx.x - mb.plan_first[i], mb.plan_first[i + 1] - mb.plan_first[i]);
}

// ---------------------------------------------------------------------------
// 3. pair bucketing
// ---------------------------------------------------------------------------

__device__ __forceinline__ void pair_bucket_range(const FrameParams &fp, const MapDev &md, uint32_t blk,
                                                  uint32_t nblk)
{
    const uint32_t P = min(md.fs->pairs.v, md.pair_cap);
    const uint32_t stride = nblk * blockDim.x;
    const bool labels = fp.K > 0 && fp.sem_kind == SLIM_IN_LABEL_I32;
    // four pairs per thread and round, each step's loads issued together
    constexpr int U = 4;
    for (uint32_t i0 = blk * blockDim.x + threadIdx.x; i0 < P; i0 += U * stride) {
        uint4 pq[U];  // (staging position, rank, key, distance bits)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * stride;
            pq[u] = i < P ? md.pairs[i] : make_uint4(kNoPos, 0u, 0u, 0u);
        }
        uint32_t dst[U];
#pragma unroll
        for (int u = 0; u < U; ++u) dst[u] = pq[u].x != kNoPos ? (uint32_t)md.pos_plan[pq[u].x].z + pq[u].y : 0u;
        int32_t lab[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            lab[u] = labels && pq[u].x != kNoPos ? point_label(fp, pq[u].z & kPidMask) : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (pq[u].x == kNoPos) continue;
            md.srt_kv[dst[u]] = make_uint2(pq[u].z, pq[u].w);
            // the leaf kernel's small items find the label beside the pair
            if (labels) md.srt_lab[dst[u]] = lab[u];
        }
    }
}

__global__ __launch_bounds__(256) void k_pair_bucket(FrameParams fp, MapDev md)
{
    pair_bucket_range(fp, md, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_pair_bucket_batch(MapBatch mb)
{
    const int i = batch_map(mb.bucket_first, mb.nmaps, blockIdx.x);
    pair_bucket_range(mb.fps[i], mb.mds[i], blockIdx.x - mb.bucket_first[i],
                      mb.bucket_first[i + 1] - mb.bucket_first[i]);
}

// ---------------------------------------------------------------------------
// 4. per-leaf sort, reduce and conjugate combine
// ---------------------------------------------------------------------------

struct LeafShared {
    uint32_t a_key[kLeafLdsPairs], b_key[kLeafLdsPairs];  // sorted / binned pairs
    float a_val[kLeafLdsPairs], b_val[kLeafLdsPairs];
    uint32_t hist[kLeafVoxels], bin0[kLeafVoxels], cur[kLeafVoxels];
    uint32_t touch[kMaskWords], occ0[kMaskWords], wsum[4];
    int pages[kLeafPages];
    uint32_t chunk_end, uold, unew;
    uint32_t stash_n;         // pairs of an x-slab item's own offsets (kept in a_key/a_val while they fit)
    uint32_t item[32];        // the current block item
};

__device__ __forceinline__ float load_emb(const FrameParams &fp, uint32_t pid, int comp)
{
    const size_t idx = (size_t)pid * fp.L + comp;
    return fp.sem_kind == SLIM_IN_EMB_BF16 ? __uint_as_float((uint32_t)((const uint16_t *)fp.sem)[idx] << 16)
                                           : ((const float *)fp.sem)[idx];
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int d = 32; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ float wave_sum(float v)
{
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Orders the wave's LDS accesses before the barrier ahead of those after it
// (lanes of one wave exchanging data through LDS).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Eq. (1)-(2) with unit weights.  Each truncated distance is taken as the
// fixed-point integer q = rint(tsdf 2^k), where 2^k is the largest power of two
// with tau 2^k <= 2^40, and a frame's q are summed in 64-bit integers: the sum
// is exact, so it does not depend on the order of the observations, and it
// differs from the real sum of the distances by at most n 2^-(k+1) (n
// observations: 2^-42 tau each), far inside the tolerance.  The running mean
// is formed in binary64 and rounded once to the stored binary32.
struct FixScale {
    float s;     // 2^k
    double inv;  // 2^-k
};

__device__ __forceinline__ FixScale fix_scale(const FrameParams &fp)
{
    int e;
    (void)frexpf(fp.tau, &e);  // tau < 2^e
    return {ldexpf(1.0f, 40 - e), ldexp(1.0, e - 40)};
}

__device__ __forceinline__ long long fix_q(float tsdf, float s) { return __float2ll_rn(tsdf * s); }

__device__ __forceinline__ long long tsdf_sum(const float *vals, uint32_t n, float s)
{
    long long sum = 0;
    for (uint32_t q = 0; q < n; ++q) sum += fix_q(vals[q], s);
    return sum;
}

__device__ __forceinline__ float tsdf_mean(float D0, float W0, float W1, long long sum, double inv)
{
    return (float)(((double)W0 * (double)D0 + (double)sum * inv) / (double)W1);
}

// One voxel, one lane: its n observations sit at keys[0..n) / vals[0..n) in
// point order.  Closed set with probability or logit rows and K <= KMAX
// classes in registers.  The record moves as 16-byte vectors.
template <int KMAX>
__device__ __forceinline__ void combine_lane(const FrameParams &fp, const MapDev &md, const uint32_t *keys,
                                             const float *vals, uint32_t n, long long rec, bool existed)
{
    static_assert(KMAX > 0, "rows of at least one class");
    constexpr int NV = (2 + KMAX + 3) / 4;
    const int nv = md.rec_stride / 4, K = fp.K;
    // up to 16 classes the record is requested first, so its round trip
    // overlaps the rows (more would spill registers)
    constexpr bool early = KMAX <= 16;
    float4 *R = (float4 *)(md.vox + (size_t)rec * md.rec_stride);
    float r[4 * NV];
    auto load_record = [&]() {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float4 x = (existed && v < nv) ? R[v] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            r[4 * v + 0] = x.x;
            r[4 * v + 1] = x.y;
            r[4 * v + 2] = x.z;
            r[4 * v + 3] = x.w;
        }
    };
    if constexpr (early) load_record();
    float acc[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) acc[k] = 0.0f;
    // the rows of RB observations are loaded before any is used (two up to 24
    // classes; more would spill registers), then each is added in point order
    constexpr int RB = KMAX <= 24 ? 2 : 1;
    for (uint32_t t0 = 0; t0 < n; t0 += RB) {
        float x[RB][KMAX];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const bool has = t0 + b < n;
            const float *row = (const float *)fp.sem + (size_t)(has ? keys[t0 + b] & kPidMask : 0u) * K;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) x[b][k] = (has && k < K) ? row[k] : 0.0f;
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            if (t0 + b < n) {
                if (fp.sem_kind == SLIM_IN_LOGIT_F32) {
                    // softmax of the logits, max-subtracted
                    float mx = x[b][0];
#pragma unroll
                    for (int k = 1; k < KMAX; ++k)
                        if (k < K) mx = fmaxf(mx, x[b][k]);
                    float den = 0.0f;
#pragma unroll
                    for (int k = 0; k < KMAX; ++k) {
                        x[b][k] = k < K ? expf(x[b][k] - mx) : 0.0f;
                        den += x[b][k];
                    }
#pragma unroll
                    for (int k = 0; k < KMAX; ++k) x[b][k] = x[b][k] / den;
                }
#pragma unroll
                for (int k = 0; k < KMAX; ++k) acc[k] += x[b][k];
            }
        }
    }
    if constexpr (!early) load_record();
    // Eq. (1)-(2) with unit weights
    const float nf = (float)n, W0 = r[1], W1 = W0 + nf;
    const FixScale fx = fix_scale(fp);
    r[0] = tsdf_mean(r[0], W0, W1, tsdf_sum(vals, n, fx.s), fx.inv);
    r[1] = W1;
    // Eq. (6): concentrations grow by the expected class counts
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (k < K) r[2 + k] += acc[k];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        if (v < nv) R[v] = make_float4(r[4 * v + 0], r[4 * v + 1], r[4 * v + 2], r[4 * v + 3]);
}

// Raw words of one lane's share of an open-set row: V / 2 words of bf16
// pairs, or V floats.
template <int V, bool BF>
struct RowWords {
    static constexpr int W = BF ? V / 2 : V;
    uint32_t w[W];
};

template <int V, bool BF>
__device__ __forceinline__ void load_row_words(const FrameParams &fp, uint32_t pid, int lane, RowWords<V, BF> &r)
{
    constexpr int W = RowWords<V, BF>::W;
    const uint32_t *row = (const uint32_t *)fp.sem + (size_t)pid * (64 * W) + lane * W;
    if constexpr (W % 4 == 0) {
#pragma unroll
        for (int c = 0; c < W / 4; ++c) {
            const uint4 u = ((const uint4 *)row)[c];
            r.w[4 * c] = u.x;
            r.w[4 * c + 1] = u.y;
            r.w[4 * c + 2] = u.z;
            r.w[4 * c + 3] = u.w;
        }
    } else if constexpr (W == 2) {
        const uint2 u = *(const uint2 *)row;
        r.w[0] = u.x;
        r.w[1] = u.y;
    } else {
#pragma unroll
        for (int c = 0; c < W; ++c) r.w[c] = row[c];
    }
}

template <int V, bool BF>
__device__ __forceinline__ void unpack_row(const RowWords<V, BF> &r, float (&z)[V])
{
    if constexpr (BF) {
#pragma unroll
        for (int e = 0; e < V / 2; ++e) {
            z[2 * e] = __uint_as_float(r.w[e] << 16);
            z[2 * e + 1] = __uint_as_float(r.w[e] & 0xFFFF0000u);
        }
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) z[e] = __uint_as_float(r.w[e]);
    }
}

// Sum over the wave of one 64-bit integer per lane (every lane gets the sum).
__device__ __forceinline__ long long wave_sum_i64(long long x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int lo = __shfl_xor((int)(unsigned long long)x, o, 64);
        const int hi = __shfl_xor((int)((unsigned long long)x >> 32), o, 64);
        x += (long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo);
    }
    return x;
}

// Open set with L = 64 V, one wave per voxel: lane l owns components l V ..
// l V + V - 1, so one observation's row is one or two wide loads per lane and
// many observations are in flight at once.  Sums as in combine_wave: the
// shifted sums in observation order, the distance sum as exact integers.  The
// point index of each row is read from its lane as a wave-uniform value, and
// a batch's rows are all requested before any is unpacked (a batch's slots
// past the last observation load that observation's row again and add
// nothing).
// kl0, vl0: point index and distance of observation `lane` (lanes below
// min(n, 64)), 0 elsewhere; the caller may have requested them ahead.
// V consecutive floats of a record (8-byte aligned for even V), read or
// written as pairs.  A record is read and written once per frame while the
// rows of the voxel's observations are read again by the neighbouring voxels:
// the record accesses are marked streaming (non-temporal), so that they do not
// push the rows out of L2.
typedef float f32x2_t __attribute__((ext_vector_type(2)));

template <int V>
__device__ __forceinline__ void rec_load(const float *p, float (&o)[V])
{
    if constexpr (V % 2 == 0) {
#pragma unroll
        for (int c = 0; c < V / 2; ++c) {
            const f32x2_t f = __builtin_nontemporal_load((const f32x2_t *)p + c);
            o[2 * c] = f.x;
            o[2 * c + 1] = f.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = __builtin_nontemporal_load(p + i);
    }
}

template <int V>
__device__ __forceinline__ void rec_store(float *p, const float (&o)[V])
{
    if constexpr (V % 2 == 0) {
#pragma unroll
        for (int c = 0; c < V / 2; ++c) {
            f32x2_t f;
            f.x = o[2 * c];
            f.y = o[2 * c + 1];
            __builtin_nontemporal_store(f, (f32x2_t *)p + c);
        }
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) __builtin_nontemporal_store(o[i], p + i);
    }
}

template <int V, bool BF>
__device__ __forceinline__ void combine_wave_vec_t(const FrameParams &fp, const MapDev &md, const uint32_t *keys,
                                                   const float *vals, uint32_t n, long long rec, bool existed,
                                                   uint32_t kl0, float vl0)
{
    // observations per batch of rows: fewer for L = 256 (few observations per
    // voxel), whose kernel runs more waves instead; a batch never crosses a
    // group of 64 observations (the lanes' point indices are reloaded there)
    constexpr int B = V >= 16 || V == 4 ? 4 : 8;
    static_assert(64 % B == 0, "batches tile the 64-observation groups");
    const int lane = lane_id();
    float *R = md.vox + (size_t)rec * md.rec_stride;
    // (up to 8 components per lane) the voxel's record is requested with the rows
    constexpr bool early = V <= 8;
    uint32_t kl = kl0;
    float vl = vl0;
    float *M = R + 2 + lane * V, *Bt = R + 2 + 64 * V + lane * V;
    float m0[early ? V : 1], b0[early ? V : 1];
    float W0 = 0.0f, D0 = 0.0f;
    if constexpr (early) {
        W0 = existed ? R[1] : 0.0f;
        D0 = existed ? R[0] : 0.0f;
        if (existed) {
            rec_load<V>(M, m0);
            rec_load<V>(Bt, b0);
        } else {
#pragma unroll
            for (int i = 0; i < V; ++i) {
                m0[i] = 0.0f;
                b0[i] = 0.0f;
            }
        }
    }
    float z0[V], s1[V], s2[V];
    {
        RowWords<V, BF> r0;
        load_row_words<V, BF>(fp, (uint32_t)__builtin_amdgcn_readlane((int)kl, 0), lane, r0);
        unpack_row<V, BF>(r0, z0);
    }
#pragma unroll
    for (int i = 0; i < V; ++i) {
        s1[i] = 0.0f;
        s2[i] = 0.0f;
    }
    // fixed-point distance sum (Eq. (1)-(2)): each lane converts its own
    // observations, one wave-wide sum at the end
    const FixScale fx = fix_scale(fp);
    long long sum_t = 0;
    // batches of B observations from observation 0 (whose difference is 0);
    // a batch never crosses a group of 64 observations
    for (uint32_t q = 0; q < n; q += B) {
        if ((q & 63u) == 0) {
            if (q > 0) {
                kl = q + (uint32_t)lane < n ? keys[q + lane] & kPidMask : 0u;
                vl = q + (uint32_t)lane < n ? vals[q + lane] : 0.0f;
            }
            if (q + (uint32_t)lane < n) sum_t += fix_q(vl, fx.s);
        }
        RowWords<V, BF> raw[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const uint32_t t = min(q + (uint32_t)b, n - 1u);
            load_row_words<V, BF>(fp, (uint32_t)__builtin_amdgcn_readlane((int)kl, (int)(t & 63u)), lane, raw[b]);
        }
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (q + b > 0 && q + b < n) {
                float z[V];
                unpack_row<V, BF>(raw[b], z);
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    const float d = z[i] - z0[i];
                    s1[i] += d;
                    s2[i] += d * d;
                }
            }
    }
    sum_t = wave_sum_i64(sum_t);
    // Eqs. (11)-(14) with lambda = W, nu = W / 2
    const float nf = (float)n;
    if constexpr (!early) {
        W0 = existed ? R[1] : 0.0f;
        D0 = existed ? R[0] : 0.0f;
    }
    const float W1 = W0 + nf;
    const float inv_n = 1.0f / nf, inv_w1 = 1.0f / W1;
    const float cross = W0 * nf * inv_w1;
    float mo[V], bo[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const float zbar = z0[i] + s1[i] * inv_n;
        const float scat = fmaxf(s2[i] - s1[i] * s1[i] * inv_n, 0.0f);
        float mi, bi;
        if constexpr (early) {
            mi = m0[i];
            bi = b0[i];
        } else {
            mi = existed ? M[i] : 0.0f;
            bi = existed ? Bt[i] : 0.0f;
        }
        const float dm = zbar - mi;
        bo[i] = bi + 0.5f * scat + cross * dm * dm * 0.5f;
        mo[i] = (W0 * mi + nf * zbar) * inv_w1;
    }
    rec_store<V>(Bt, bo);
    rec_store<V>(M, mo);
    if (lane == 0) {
        R[0] = tsdf_mean(D0, W0, W1, sum_t, fx.inv);
        R[1] = W1;
    }
}

template <int V>
__device__ __forceinline__ void combine_wave_vec(const FrameParams &fp, const MapDev &md, const uint32_t *keys,
                                                 const float *vals, uint32_t n, long long rec, bool existed,
                                                 uint32_t kl0, float vl0)
{
    if constexpr (V >= 2) {
        if (fp.sem_kind == SLIM_IN_EMB_BF16) {
            combine_wave_vec_t<V, true>(fp, md, keys, vals, n, rec, existed, kl0, vl0);
            return;
        }
    }
    combine_wave_vec_t<V, false>(fp, md, keys, vals, n, rec, existed, kl0, vl0);
}

template <int V>
__device__ __forceinline__ void combine_wave_vec(const FrameParams &fp, const MapDev &md, const uint32_t *keys,
                                                 const float *vals, uint32_t n, long long rec, bool existed)
{
    const uint32_t lane = (uint32_t)lane_id();
    combine_wave_vec<V>(fp, md, keys, vals, n, rec, existed, lane < n ? keys[lane] & kPidMask : 0u,
                        lane < n ? vals[lane] : 0.0f);
}

constexpr int kWaveComps = 16;
constexpr int kWaveBatch = 4;  // observations whose rows are in flight at once

// One voxel, one wave: lane l owns components l, l + 64, ... of the open-set
// statistics (L <= 1024) or of the class counts (K <= 1024).  The rows of
// kWaveBatch observations are loaded before any is used.  Open set: one pass
// over the observations with sums shifted by the first one, s1 = sum (z - z_0),
// s2 = sum (z - z_0)^2, so the batch mean is z_0 + s1 / n and the scatter
// s2 - s1^2 / n (the shift keeps the subtraction well conditioned).
__device__ __forceinline__ void combine_wave(const FrameParams &fp, const MapDev &md, const uint32_t *keys,
                                             const float *vals, uint32_t n, long long rec, bool existed)
{
    const int lane = lane_id();
    const bool open = fp.L > 0;
    const int C = open ? fp.L : fp.K;
    float *R = md.vox + (size_t)rec * md.rec_stride;
    float s1[kWaveComps], s2[kWaveComps];
#pragma unroll
    for (int j = 0; j < kWaveComps; ++j) {
        s1[j] = 0.0f;
        s2[j] = 0.0f;
    }
    // the point indices of 64 observations at a time, one per lane; a batch's
    // indices come from the lanes, so its rows do not wait on a load of them
    // (batches start at multiples of their size and never cross a window)
    uint32_t kl = (uint32_t)lane < n ? keys[lane] & kPidMask : 0u;
    auto window = [&](uint32_t q) {
        if (q > 0 && (q & 63u) == 0) kl = q + (uint32_t)lane < n ? keys[q + lane] & kPidMask : 0u;
    };
    auto pid_at = [&](uint32_t t) { return (uint32_t)__shfl((int)kl, (int)(t & 63u), 64); };
    if (open) {
        float z0[kWaveComps];
        const uint32_t p0 = pid_at(0);
#pragma unroll
        for (int j = 0; j < kWaveComps; ++j) z0[j] = (lane + 64 * j < C) ? load_emb(fp, p0, lane + 64 * j) : 0.0f;
        // observation 0 enters as its own difference, 0
        for (uint32_t q = 0; q < n; q += kWaveBatch) {
            window(q);
            float z[kWaveBatch][kWaveComps];
#pragma unroll
            for (int b = 0; b < kWaveBatch; ++b) {
                const bool has = q + b < n && q + b > 0;
                const uint32_t pid = pid_at(q + b);
#pragma unroll
                for (int j = 0; j < kWaveComps; ++j)
                    z[b][j] = (has && lane + 64 * j < C) ? load_emb(fp, pid, lane + 64 * j) : z0[j];
            }
#pragma unroll
            for (int b = 0; b < kWaveBatch; ++b)
#pragma unroll
                for (int j = 0; j < kWaveComps; ++j) {
                    const float d = z[b][j] - z0[j];
                    s1[j] += d;
                    s2[j] += d * d;
                }
        }
        // Eqs. (11)-(14) with lambda = W, nu = W / 2
        const float nf = (float)n;
        const float W0 = existed ? R[1] : 0.0f, W1 = W0 + nf;
        const float inv_n = 1.0f / nf, inv_w1 = 1.0f / W1;
        const float cross = W0 * nf * inv_w1;
        float *M = R + 2, *B = R + 2 + fp.L;
#pragma unroll
        for (int j = 0; j < kWaveComps; ++j) {
            const int comp = lane + 64 * j;
            if (comp < C) {
                const float zbar = z0[j] + s1[j] * inv_n;
                const float scat = fmaxf(s2[j] - s1[j] * s1[j] * inv_n, 0.0f);
                const float m0 = existed ? M[comp] : 0.0f, b0 = existed ? B[comp] : 0.0f;
                const float dm = zbar - m0;
                B[comp] = b0 + 0.5f * scat + cross * dm * dm * 0.5f;
                M[comp] = (W0 * m0 + nf * zbar) * inv_w1;
            }
        }
    } else if (fp.sem_kind == SLIM_IN_LABEL_I32) {
        for (uint32_t q = 0; q < n; q += 2 * kWaveBatch) {
            window(q);
            int lab[2 * kWaveBatch];
#pragma unroll
            for (int b = 0; b < 2 * kWaveBatch; ++b) {
                const uint32_t pid = pid_at(q + b);
                lab[b] = q + b < n ? ((const int32_t *)fp.sem)[pid] : -1;
            }
#pragma unroll
            for (int b = 0; b < 2 * kWaveBatch; ++b)
#pragma unroll
                for (int j = 0; j < kWaveComps; ++j) s1[j] += (lab[b] == lane + 64 * j) ? 1.0f : 0.0f;
        }
    } else if (fp.sem_kind == SLIM_IN_PROB_F32) {
        for (uint32_t q = 0; q < n; q += kWaveBatch) {
            window(q);
            float x[kWaveBatch][kWaveComps];
#pragma unroll
            for (int b = 0; b < kWaveBatch; ++b) {
                const bool has = q + b < n;
                const uint32_t pid = pid_at(q + b);
                const size_t row = has ? (size_t)pid * C : 0;
#pragma unroll
                for (int j = 0; j < kWaveComps; ++j)
                    x[b][j] = (has && lane + 64 * j < C) ? ((const float *)fp.sem)[row + lane + 64 * j] : 0.0f;
            }
#pragma unroll
            for (int b = 0; b < kWaveBatch; ++b)
#pragma unroll
                for (int j = 0; j < kWaveComps; ++j) s1[j] += x[b][j];
        }
    } else {
        // logits, K <= 64: softmax across the wave
        for (uint32_t q = 0; q < n; q += kWaveBatch) {
            window(q);
            float l[kWaveBatch];
#pragma unroll
            for (int b = 0; b < kWaveBatch; ++b) {
                const uint32_t pid = pid_at(q + b);
                l[b] = (q + b < n && lane < C) ? ((const float *)fp.sem)[(size_t)pid * C + lane] : -INFINITY;
            }
#pragma unroll
            for (int b = 0; b < kWaveBatch; ++b) {
                if (q + b >= n) break;
                const float mx = wave_max(l[b]);
                const float e = lane < C ? expf(l[b] - mx) : 0.0f;
                s1[0] += e / wave_sum(e);
            }
        }
    }
    const float nf = (float)n;
    const float W0 = existed ? R[1] : 0.0f, W1 = W0 + nf;
    const float D0 = existed ? R[0] : 0.0f;
    if (!open) {
#pragma unroll
        for (int j = 0; j < kWaveComps; ++j) {
            const int comp = lane + 64 * j;
            if (comp < C) R[2 + comp] = (existed ? R[2 + comp] : 0.0f) + s1[j];
        }
    }
    // fixed-point distance sum, 64 distances loaded at a time, one per lane
    const FixScale fx = fix_scale(fp);
    long long sum_t = 0;
    for (uint32_t w0 = 0; w0 < n; w0 += 64)
        sum_t += w0 + (uint32_t)lane < n ? fix_q(vals[w0 + lane], fx.s) : 0ll;
    for (int d = 32; d > 0; d >>= 1) sum_t += __shfl_xor(sum_t, d, 64);
    if (lane == 0) {
        R[0] = tsdf_mean(D0, W0, W1, sum_t, fx.inv);
        R[1] = W1;
    }
}

// Non-Bayesian mode (SLIM-VDB*, Sec. IV): D and W as Eq. (1)-(2); the voxel's
// semantics become those of its most recent measurement, the last pair in point
// order (a ray visits a voxel at most once, so point indices are distinct).
// Closed set, one lane per voxel: the class the measurement names -- its label,
// or the first index of the largest probability or logit of its row.
__device__ __forceinline__ void combine_last_lane(const FrameParams &fp, const MapDev &md, const uint32_t *keys,
                                                  const float *vals, uint32_t n, long long rec, bool existed)
{
    const uint32_t pid = keys[n - 1] & kPidMask;
    int cls;
    if (fp.sem_kind == SLIM_IN_LABEL_I32) {
        cls = ((const int32_t *)fp.sem)[pid];
    } else {
        const float *row = (const float *)fp.sem + (size_t)pid * fp.K;
        float best = row[0];
        cls = 0;
        for (int k = 1; k < fp.K; ++k) {
            const float x = row[k];
            if (x > best) {
                best = x;
                cls = k;
            }
        }
    }
    float4 *R = (float4 *)(md.vox + (size_t)rec * md.rec_stride);
    const float4 r = existed ? R[0] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float nf = (float)n, W1 = r.y + nf;
    const FixScale fx = fix_scale(fp);
    R[0] = make_float4(tsdf_mean(r.x, r.y, W1, tsdf_sum(vals, n, fx.s), fx.inv), W1, (float)cls, 0.0f);
}

// Open set, one wave per voxel: lane l copies components l, l + 64, ... of the
// measurement's embedding.
__device__ __forceinline__ void combine_last_wave(const FrameParams &fp, const MapDev &md, const uint32_t *keys,
                                                  const float *vals, uint32_t n, long long rec, bool existed)
{
    const uint32_t pid = keys[n - 1] & kPidMask;
    float *R = md.vox + (size_t)rec * md.rec_stride;
    for (int comp = lane_id(); comp < fp.L; comp += 64) R[2 + comp] = load_emb(fp, pid, comp);
    if (lane_id() == 0) {
        const float W0 = existed ? R[1] : 0.0f, D0 = existed ? R[0] : 0.0f, W1 = W0 + (float)n;
        const FixScale fx = fix_scale(fp);
        R[0] = tsdf_mean(D0, W0, W1, tsdf_sum(vals, n, fx.s), fx.inv);
        R[1] = W1;
    }
}

// Combines every touched voxel with offset in [o0, o1); the sorted pairs of
// bin o sit at keys[bin0[o] - base] / vals[bin0[o] - base] (LDS or global).
// Bits of touched-mask word w that fall in offsets [o0, o1).
__device__ __forceinline__ uint32_t range_bits(uint32_t bits, uint32_t w, uint32_t o0, uint32_t o1)
{
    if ((w << 5) < o0) bits &= ~0u << (o0 & 31);
    if (((w + 1) << 5) > o1) bits &= (o1 & 31) ? ((1u << (o1 & 31)) - 1u) : ~0u;
    return bits;
}

// Position of the k-th set bit (from 0) of x, which has more than k set bits.
__device__ __forceinline__ uint32_t select_bit(uint32_t x, uint32_t k)
{
    uint32_t pos = 0;
#pragma unroll
    for (int s = 16; s > 0; s >>= 1) {
        const uint32_t low = x & ((1u << s) - 1u), c = (uint32_t)__popc(low);
        if (k >= c) {
            k -= c;
            x >>= s;
            pos += (uint32_t)s;
        } else {
            x = low;
        }
    }
    return pos;
}

template <int KMAX, bool WAVE, bool ROWS>
__device__ void combine_range(const FrameParams &fp, const MapDev &md, LeafShared &sh, const uint32_t *keys,
                              const float *vals, uint32_t o0, uint32_t o1, uint32_t base)
{
    if constexpr (!WAVE) {
        // thread t takes the touched offsets of rank t, t + blockDim.x, ... in
        // [o0, o1), so a leaf with at most blockDim.x touched voxels loads its
        // records in one round
        const uint32_t w0 = o0 >> 5, w1 = (o1 - 1) >> 5;
        uint32_t cnt = 0;
        for (uint32_t w = w0; w <= w1; ++w) cnt += __popc(range_bits(sh.touch[w], w, o0, o1));
        for (uint32_t r = threadIdx.x; r < cnt; r += blockDim.x) {
            uint32_t w = w0, before = 0, bits = 0;
            for (; w <= w1; ++w) {
                bits = range_bits(sh.touch[w], w, o0, o1);
                const uint32_t c = __popc(bits);
                if (r < before + c) break;
                before += c;
            }
            const uint32_t o = (w << 5) + select_bit(bits, r - before);
            const uint32_t n = sh.hist[o];
            const long long rec = (long long)sh.pages[o >> 6] * kPageVoxels + (o & (kPageVoxels - 1));
            const bool existed = (sh.occ0[o >> 5] >> (o & 31)) & 1u;
            if constexpr (KMAX < 0)
                combine_last_lane(fp, md, keys + (sh.bin0[o] - base), vals + (sh.bin0[o] - base), n, rec, existed);
            else
                combine_lane<KMAX>(fp, md, keys + (sh.bin0[o] - base), vals + (sh.bin0[o] - base), n, rec, existed);
        }
    } else {
        const uint32_t wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
        for (uint32_t o = o0 + wave; o < o1; o += nw) {
            const uint32_t n = sh.hist[o];
            if (!n) continue;
            const long long rec = (long long)sh.pages[o >> 6] * kPageVoxels + (o & (kPageVoxels - 1));
            const bool existed = (sh.occ0[o >> 5] >> (o & 31)) & 1u;
            if (KMAX < 0)
                combine_last_wave(fp, md, keys + (sh.bin0[o] - base), vals + (sh.bin0[o] - base), n, rec, existed);
            else if (KMAX > 0)  // wave kernels: KMAX is the components per lane of a word-aligned embedding
                combine_wave_vec<(KMAX > 0 ? KMAX : 1)>(fp, md, keys + (sh.bin0[o] - base), vals + (sh.bin0[o] - base),
                                                        n, rec, existed);
            else
                combine_wave(fp, md, keys + (sh.bin0[o] - base), vals + (sh.bin0[o] - base), n, rec, existed);
        }
    }
}

// Orders the pairs of bins [o0, o1) (binned in `bk`/`bv`, at bucket indices
// starting at `lo`) by point index inside each bin: a pair's position is the
// number of smaller keys in its bin.  Writes sh.a_*.
template <class KP, class VP>
__device__ __forceinline__ void rank_bins(LeafShared &sh, KP bk, VP bv, uint32_t lo, uint32_t hi)
{
    for (uint32_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
        const uint32_t k = bk[t - lo];
        const uint32_t o = k >> kPidBits, blo = sh.bin0[o], bhi = blo + sh.hist[o];
        uint32_t r = 0;
#pragma unroll 8
        for (uint32_t u = blo; u < bhi; ++u) r += bk[u - lo] < k;
        sh.a_key[blo + r - lo] = k;
        sh.a_val[blo + r - lo] = bv[t - lo];
    }
}

// One work item of the leaf kernel: the touched leaf of item *itp, all
// of it (slab < 0) or, for a leaf with more pairs than LDS holds, the voxels
// of one x-slab (offsets 64 slab .. 64 slab + 63), so that the slabs of a
// large leaf run in different workgroups.  Reads every pair of the leaf for
// the offset histogram (which fixes the bucket position of every voxel),
// keeps those of its offsets, orders them by point index inside each voxel and
// combines the voxels.  An x-slab item reads the leaf once when its own pairs
// fit LDS and a second time otherwise.
template <int KMAX, bool WAVE, bool ROWS>
__device__ __forceinline__ void fuse_item(const FrameParams &fp, const MapDev &md, LeafShared &sh, LeafItem *itp,
                                          int slab, unsigned long long lused, bool ok)
{
    const int tid = threadIdx.x;
    if (tid < 32) sh.item[tid] = ((const uint32_t *)itp)[tid];
    for (int o = tid; o < kLeafVoxels; o += blockDim.x) sh.hist[o] = 0;
    if (tid == 0) sh.stash_n = 0;
    __syncthreads();
    const uint32_t pos = sh.item[0], n = sh.item[1], bstart = sh.item[2];
    const int islot = (int)sh.item[3];
    const int slot = islot >= 0 ? islot : (int)(lused + (unsigned long long)(-1 - islot));
    const uint32_t ob = slab < 0 ? 0u : 64u * (uint32_t)slab, oe = slab < 0 ? (uint32_t)kLeafVoxels : ob + 64u;
    // a new leaf is inserted by the item of its lowest touched slab (or its
    // whole-leaf item); the first probe goes out with the pair loads
    const bool lead = slab < 0 || (uint32_t)slab == (uint32_t)(__ffs(sh.item[4] & 0xFFu) - 1);
    const bool inserts = ok && lead && islot < 0 && tid == 0;
    const unsigned long long lkey = ((unsigned long long)sh.item[7] << 32) | sh.item[6];
    uint32_t ih = 0;
    unsigned long long iprev = 0;
    if (inserts) iprev = map_insert_start(md, lkey, &ih);
    if (tid < kMaskWords) sh.occ0[tid] = sh.item[16 + tid];
    if (tid < kLeafPages) sh.pages[tid] = (int)sh.item[8 + tid];

    const uint2 *gkv = md.srt_kv + bstart;
    uint32_t *tk = md.tmp_key + bstart;
    float *tv = md.tmp_tsdf + bstart;
    const bool whole_small = slab < 0 && n <= (uint32_t)kLeafLdsPairs;

    // histogram of the voxel offsets of every pair of the leaf; kLeafBatch loads
    // in flight per thread, and a whole leaf that fits LDS stays in registers
    uint32_t rk[kLeafBatch];
    float rv[kLeafBatch];
    if (whole_small) {
#pragma unroll
        for (int u = 0; u < kLeafBatch; ++u) {
            const uint32_t t = u * kLeafThreads + tid;
            const uint2 e = t < n ? gkv[t] : make_uint2(0u, 0u);
            rk[u] = e.x;
            rv[u] = __uint_as_float(e.y);
        }
#pragma unroll
        for (int u = 0; u < kLeafBatch; ++u)
            if ((uint32_t)(u * kLeafThreads + tid) < n) atomicAdd(&sh.hist[rk[u] >> kPidBits], 1u);
    } else {
        // every pair into the histogram; the pairs of the item's own offsets
        // into a_key/a_val in arrival order, as long as they fit (one slot
        // reservation per wave and batch)
        for (uint32_t t0 = 0; t0 < n; t0 += kLeafLdsPairs) {
#pragma unroll
            for (int u = 0; u < kLeafBatch; ++u) {
                const uint32_t t = t0 + u * kLeafThreads + tid;
                const uint2 e = t < n ? gkv[t] : make_uint2(0u, 0u);
                rk[u] = e.x;
                rv[u] = __uint_as_float(e.y);
            }
            uint32_t mine = 0;
#pragma unroll
            for (int u = 0; u < kLeafBatch; ++u) {
                const uint32_t o = rk[u] >> kPidBits;
                if (t0 + u * kLeafThreads + tid < n) {
                    atomicAdd(&sh.hist[o], 1u);
                    mine += (o >= ob && o < oe) ? 1u : 0u;
                }
            }
            const uint32_t incl = wave_incl_scan(mine);
            uint32_t wbase = 0;
            if (lane_id() == 63 && incl) wbase = atomicAdd(&sh.stash_n, incl);
            uint32_t q = __shfl(wbase, 63, 64) + incl - mine;
#pragma unroll
            for (int u = 0; u < kLeafBatch; ++u) {
                const uint32_t o = rk[u] >> kPidBits;
                if (t0 + u * kLeafThreads + tid < n && o >= ob && o < oe) {
                    if (q < (uint32_t)kLeafLdsPairs) {
                        sh.a_key[q] = rk[u];
                        sh.a_val[q] = rv[u];
                    }
                    q++;
                }
            }
        }
    }
    __syncthreads();
    block_scan512(sh.hist, sh.bin0, sh.wsum);
    for (int o = tid; o < kLeafVoxels; o += blockDim.x) sh.cur[o] = sh.bin0[o];
    {
        // touched offsets: wave w covers bins 64w + [0, 64) and 256 + 64w + [0, 64)
        const int w = tid >> 6;
        const unsigned long long b0 = __ballot(sh.hist[tid] != 0u);
        const unsigned long long b1 = __ballot(sh.hist[tid + 256] != 0u);
        if (lane_id() == 0) {
            sh.touch[2 * w] = (uint32_t)b0;
            sh.touch[2 * w + 1] = (uint32_t)(b0 >> 32);
            sh.touch[8 + 2 * w] = (uint32_t)b1;
            sh.touch[9 + 2 * w] = (uint32_t)(b1 >> 32);
        }
    }
    __syncthreads();
    if (WAVE && ok && lead) {
        // the leaf's item that inserts it also lists all its touched voxels for
        // the wave combine, in offset order at consecutive entries, so that the
        // voxels of one leaf (which share observations) are combined at the
        // same time; every item of the leaf has its histogram, so the voxel's
        // sorted pairs start at bucket position bin0[o] whichever item sorts them
        if (tid == 0) {
            uint32_t t = 0;
            for (int q = 0; q < kMaskWords; ++q) t += __popc(sh.touch[q]);
            sh.chunk_end = atomicAdd(&md.fs->n_vox.v, t);  // (free until the runs below)
        }
        __syncthreads();
        const uint32_t vbase = sh.chunk_end;
        for (uint32_t o = tid; o < (uint32_t)kLeafVoxels; o += blockDim.x) {
            const uint32_t n_o = sh.hist[o];
            if (!n_o) continue;
            // rank of o among the leaf's touched offsets
            uint32_t r = __popc(sh.touch[o >> 5] & ((1u << (o & 31)) - 1u));
            for (uint32_t w32 = 0; w32 < (o >> 5); ++w32) r += __popc(sh.touch[w32]);
            const uint32_t rec = (uint32_t)sh.pages[o >> 6] * kPageVoxels + (o & (kPageVoxels - 1));
            const uint32_t existed = (sh.occ0[o >> 5] >> (o & 31)) & 1u;
            md.vox_list[vbase + r] = make_uint4(rec, n_o | (existed << 31), bstart + sh.bin0[o], 0u);
        }
    }
    const uint32_t lo_all = sh.bin0[ob], hi_all = oe < (uint32_t)kLeafVoxels ? sh.bin0[oe] : n;
    const bool small = whole_small || (slab >= 0 && hi_all - lo_all <= (uint32_t)kLeafLdsPairs);
    if (tid == 0) {
        uint32_t uo = 0, un = 0;
        for (uint32_t w = ob >> 5; w < (oe >> 5); ++w) {
            uo += __popc(sh.touch[w] & sh.occ0[w]);
            un += __popc(sh.touch[w] & ~sh.occ0[w]);
        }
        sh.uold += uo;
        sh.unew += un;
    }

    // bin by offset (order inside a bin arbitrary): in LDS if the item fits,
    // else in the scratch buffer.  An x-slab item that fits bins from the
    // pairs it kept (exactly those of its offsets: their count is the width
    // of its range of the histogram)
    if (whole_small) {
#pragma unroll
        for (int u = 0; u < kLeafBatch; ++u)
            if ((uint32_t)(u * kLeafThreads + tid) < n) {
                const uint32_t p = atomicAdd(&sh.cur[rk[u] >> kPidBits], 1u);
                sh.b_key[p] = rk[u];
                sh.b_val[p] = rv[u];
            }
    } else if (small) {
        const uint32_t m = hi_all - lo_all;
        for (uint32_t t = tid; t < m; t += blockDim.x) {
            const uint32_t k = sh.a_key[t];
            const uint32_t p = atomicAdd(&sh.cur[k >> kPidBits], 1u);
            sh.b_key[p - lo_all] = k;
            sh.b_val[p - lo_all] = sh.a_val[t];
        }
    } else {
        for (uint32_t t0 = 0; t0 < n; t0 += kLeafLdsPairs) {
#pragma unroll
            for (int u = 0; u < kLeafBatch; ++u) {
                const uint32_t t = t0 + u * kLeafThreads + tid;
                const uint2 e = t < n ? gkv[t] : make_uint2(0u, 0u);
                rk[u] = e.x;
                rv[u] = __uint_as_float(e.y);
            }
#pragma unroll
            for (int u = 0; u < kLeafBatch; ++u) {
                const uint32_t o = rk[u] >> kPidBits;
                if (t0 + u * kLeafThreads + tid < n && o >= ob && o < oe) {
                    const uint32_t p = atomicAdd(&sh.cur[o], 1u);
                    tk[p] = rk[u];
                    tv[p] = rv[u];
                }
            }
        }
    }
    __syncthreads();

    // runs of whole bins that fit LDS: order each bin by point index, then
    // combine its voxels (a small item is one run, already in LDS)
    uint32_t o0 = ob;
    while (o0 < oe) {
        uint32_t o1 = oe;
        if (!small) {
            if (tid == 0) {
                // bin ends are non-decreasing: first o1 > o0 whose end passes
                // bin0[o0] + capacity (at least o0 + 1)
                const uint32_t lim = sh.bin0[o0] + (uint32_t)kLeafLdsPairs;
                uint32_t lo = o0 + 1, hi = oe;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (sh.bin0[mid] + sh.hist[mid] <= lim) lo = mid + 1;
                    else hi = mid;
                }
                sh.chunk_end = lo;
            }
            __syncthreads();
            o1 = sh.chunk_end;
        }
        const uint32_t lo = sh.bin0[o0], hi = (o1 < (uint32_t)kLeafVoxels) ? sh.bin0[o1] : n;
        const bool fits = hi - lo <= (uint32_t)kLeafLdsPairs;
        if (fits) {
            if (!small) {
                for (uint32_t t = lo + tid; t < hi; t += blockDim.x) {
                    sh.b_key[t - lo] = tk[t];
                    sh.b_val[t - lo] = tv[t];
                }
                __syncthreads();
            }
            rank_bins(sh, sh.b_key, sh.b_val, lo, hi);
        } else {
            // one bin larger than LDS: order it into the walk's pair buffers
            // (consumed by the bucketing, free now), at the bin's own range of
            // the leaf's bucket, which no other item touches
            uint32_t *bk = md.pair_key + bstart;
            float *bv = md.pair_tsdf + bstart;
            for (uint32_t t = lo + tid; t < hi; t += blockDim.x) {
                const uint32_t k = tk[t];
                uint32_t r = 0;
                for (uint32_t u = lo; u < hi; ++u) r += tk[u] < k;
                bk[lo + r] = k;
                bv[lo + r] = tv[t];
            }
        }
        __syncthreads();
        if (ok && WAVE) {
            // wave combines run in their own kernel over every voxel of the frame:
            // the sorted pairs go to the pair buffers at their bucket positions
            if (fits)
                for (uint32_t t = tid; t < hi - lo; t += blockDim.x) {
                    md.pair_key[bstart + lo + t] = sh.a_key[t];
                    md.pair_tsdf[bstart + lo + t] = sh.a_val[t];
                }
        } else if (ok) {
            // sorted pairs of bin o sit at keys[bin0[o] - base]
            const uint32_t *ck = fits ? sh.a_key : md.pair_key + bstart;
            const float *cv = fits ? sh.a_val : md.pair_tsdf + bstart;
            combine_range<KMAX, WAVE, ROWS>(fp, md, sh, ck, cv, o0, o1, fits ? lo : 0u);
        }
        __syncthreads();
        o0 = o1;
    }

    // leaf bookkeeping: an item owns the page entry and the occupancy words of
    // its offsets; the item of the leaf's lowest touched slab (or the whole-leaf
    // item) also inserts a new leaf and writes the entries of untouched slabs
    if (ok) {
        const uint32_t tslabs = sh.item[4] & 0xFFu;
        if (inserts) {
            map_insert_finish(md, lkey, slot, ih, iprev);
            md.leaf_key[slot] = lkey;
        }
        if (tid < kLeafPages) {
            const bool mine = slab < 0 || tid == slab || (lead && !((tslabs >> tid) & 1u));
            if (mine) md.leaf_page[(size_t)slot * kLeafPages + tid] = sh.pages[tid];
        }
        if (tid < kMaskWords) {
            const int sl = tid >> 1;
            const bool mine = slab < 0 || sl == slab || (lead && !((tslabs >> sl) & 1u));
            if (mine) md.leaf_occ[(size_t)slot * kMaskWords + tid] = sh.occ0[tid] | sh.touch[tid];
        }
    }
    __syncthreads();
    if (tid == 0) {
        // the staging entry is clean for the next frame once the leaf's last
        // item is done (a whole-leaf item is the only one; slab items count
        // themselves in the item's spare word, which the plan kernel zeroes)
        const bool last = slab < 0 || atomicAdd(&itp->pad, 1u) + 1u == (uint32_t)__popc(sh.item[4] & 0xFFu);
        if (last) {
            md.skeys[pos] = kEmptyKey;
            md.pos_count[pos] = 0u;
            md.pos_slab[pos] = 0u;
        }
    }
}

// A touched leaf with at most kWaveItemPairs pairs is the work of one wave:
// its pairs are ordered in the wave's quarter of the block's LDS by the full
// key (offset, point index), which groups them by voxel in point order; lanes
// then take one voxel each.  Waves run such leaves independently (no block
// barrier), four per block.
constexpr int kWaveLds = kLeafLdsPairs / 4;  // LDS pairs per wave
static_assert(kWaveItemPairs <= kWaveLds, "a wave item must fit its LDS quarter");

template <int KMAX, bool WAVE, bool ROWS>
__device__ __forceinline__ void fuse_wave_item(const FrameParams &fp, const MapDev &md, LeafShared &sh,
                                               const LeafItem *itp, unsigned long long lused, bool ok)
{
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t *wk = sh.a_key + w * kWaveLds;
    float *wv = sh.a_val + w * kWaveLds;
    uint32_t *seg = sh.b_key + w * kWaveLds;     // voxel segment starts
    uint32_t *wt = sh.hist + w * 16;             // touched-offset mask (16 words)
    uint32_t *wo = sh.bin0 + w * 16;             // occupancy words of the leaf before this frame
    int *wp = (int *)sh.cur + w * 8;             // record pages of the leaf's slabs
    uint32_t *wi = sh.cur + 64 + w * 32;         // the leaf's item
    if (lane < 32) wi[lane] = ((const uint32_t *)itp)[lane];
    wave_sync();
    const uint32_t pos = wi[0], n = wi[1], bstart = wi[2];
    const int islot = (int)wi[3];
    const int slot = islot >= 0 ? islot : (int)(lused + (unsigned long long)(-1 - islot));
    // a new leaf's first insertion probe goes out with the pair loads
    const bool inserts = ok && islot < 0 && lane == 0;
    const unsigned long long lkey = ((unsigned long long)wi[7] << 32) | wi[6];
    uint32_t ih = 0;
    unsigned long long iprev = 0;
    if (inserts) iprev = map_insert_start(md, lkey, &ih);
    // the pairs in registers (four per lane), their keys also in LDS; keys are
    // distinct (a ray visits a voxel once), so a pair's rank is the number of
    // smaller keys, and writing each pair at its rank sorts them by (offset,
    // point index)
    uint32_t *uk = sh.b_key + w * kWaveLds;  // unsorted keys, padded to a multiple of 4
    uint32_t kq[4];
    float vq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = lane + 64 * q;
        const bool has = i < n;
        const uint2 e = has ? md.srt_kv[bstart + i] : make_uint2(0xFFFFFFFFu, 0u);
        kq[q] = e.x;
        vq[q] = __uint_as_float(e.y);
        if (i < ((n + 3u) & ~3u)) uk[i] = kq[q];
    }
    const uint32_t occ = lane < kMaskWords ? wi[16 + lane] : 0u;
    const int page = lane < kLeafPages ? (int)wi[8 + lane] : -1;
    if (lane < 16) {
        wt[lane] = 0u;
        wo[lane] = occ;
    }
    if (lane < kLeafPages) wp[lane] = page;
    wave_sync();
    uint32_t rq[4] = {0u, 0u, 0u, 0u};
    for (uint32_t s4 = 0; s4 < n; s4 += 4) {
        const uint4 c = *(const uint4 *)(uk + s4);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            rq[q] += (uint32_t)(c.x < kq[q]) + (uint32_t)(c.y < kq[q]) + (uint32_t)(c.z < kq[q]) +
                     (uint32_t)(c.w < kq[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (lane + 64 * q < n) {
            wk[rq[q]] = kq[q];
            wv[rq[q]] = vq[q];
        }
    wave_sync();
    // voxel segments: starts where the offset changes
    uint32_t nseg = 0;
    const uint32_t per = (n + 63u) >> 6;
    for (uint32_t q = 0; q < per; ++q) {
        const uint32_t i = lane + 64 * q;
        const bool start = i < n && (i == 0 || (wk[i] >> kPidBits) != (wk[i - 1] >> kPidBits));
        const unsigned long long b = __ballot(start);
        if (start) seg[nseg + __popcll(b & ((1ull << lane) - 1ull))] = i;
        nseg += (uint32_t)__popcll(b);
    }
    wave_sync();
    for (uint32_t sgi = lane; sgi < nseg; sgi += 64) {
        const uint32_t o = wk[seg[sgi]] >> kPidBits;
        atomicOr(&wt[o >> 5], 1u << (o & 31));
    }
    wave_sync();
    if (ok) {
        for (uint32_t sgi = lane; sgi < nseg; sgi += 64) {
            const uint32_t b0 = seg[sgi], b1 = sgi + 1 < nseg ? seg[sgi + 1] : n;
            const uint32_t o = wk[b0] >> kPidBits;
            const int pg = wp[o >> 6];
            const uint32_t ow = wo[o >> 5];
            const long long rec = (long long)pg * kPageVoxels + (o & (kPageVoxels - 1));
            const bool existed = (ow >> (o & 31)) & 1u;
            if constexpr (KMAX < 0)
                combine_last_lane(fp, md, wk + b0, wv + b0, b1 - b0, rec, existed);
            else
                combine_lane<KMAX>(fp, md, wk + b0, wv + b0, b1 - b0, rec, existed);
        }
    }
    // statistics and leaf bookkeeping
    const uint32_t tw = lane < kMaskWords ? wt[lane] : 0u;
    uint32_t uo = __popc(tw & occ), un = __popc(tw & ~occ);
    for (int d = 32; d > 0; d >>= 1) {
        uo += __shfl_xor(uo, d, 64);
        un += __shfl_xor(un, d, 64);
    }
    if (lane == 0) {
        atomicAdd(&sh.uold, uo);
        atomicAdd(&sh.unew, un);
    }
    if (ok) {
        if (inserts) {
            map_insert_finish(md, lkey, slot, ih, iprev);
            md.leaf_key[slot] = lkey;
        }
        if (lane < kLeafPages) md.leaf_page[(size_t)slot * kLeafPages + lane] = page;
        if (lane < kMaskWords) md.leaf_occ[(size_t)slot * kMaskWords + lane] = occ | tw;
    }
    if (lane == 0) {
        md.skeys[pos] = kEmptyKey;
        md.pos_count[pos] = 0u;
        md.pos_slab[pos] = 0u;
    }
    wave_sync();
}

// The leaf kernel's work of one map's frame for blocks blk, blk + nblk, ...:
// first the slab items of large leaves (the longest work, started first), then
// every other touched leaf whole.  Block statistics go to md.blk_stats[blk].
template <int KMAX, bool WAVE, bool ROWS>
__device__ __forceinline__ void leaf_fuse_range(const FrameParams &fp, const MapDev &md, LeafShared &sh,
                                                uint32_t blk, uint32_t nblk)
{
    const DevState *st = md.st;
    const uint32_t nbig = min(md.fs->work_big.v, md.work_cap);
    const unsigned long long lused = st->leaves_used;
    const bool ok = md.fs->frame_err.v == 0 && st->pass_failed == 0 &&
                    lused + md.fs->new_leaves.v <= (unsigned long long)md.max_leaves &&
                    st->pages_used + md.fs->new_pages.v <= (unsigned long long)md.max_pages;
    if (threadIdx.x == 0) {
        sh.uold = 0;
        sh.unew = 0;
    }
    __syncthreads();
    // units of work, one per block at a time: the slab items of large leaves,
    // then the leaves done by a workgroup, then groups of four small leaves
    // (one per wave; the wave kernels take the small leaves one per workgroup)
    // each list: its larger leaves from the front of the array, then its
    // smaller ones from the back
    const uint32_t medf = (uint32_t)md.fs->n_lists, smallf = (uint32_t)(md.fs->n_lists >> 32);
    const uint32_t nmed = medf + (uint32_t)md.fs->n_lists_tail;
    const uint32_t nsmall = smallf + (uint32_t)(md.fs->n_lists_tail >> 32);
    const uint32_t last = md.hmask;
    auto med_at = [&](uint32_t m) { return &md.items[m < medf ? m : last - (m - medf)]; };
    auto small_at = [&](uint32_t k) { return &md.items_small[k < smallf ? k : last - (k - smallf)]; };
    const uint32_t nw = blockDim.x >> 6, w = threadIdx.x >> 6;
    const uint32_t ngroups = WAVE ? nsmall : (nsmall + nw - 1) / nw;
    const uint32_t nunits = nbig + nmed + ngroups;
    for (uint32_t u = blk; u < nunits; u += nblk) {
        if (u < nbig) {
            const int2 it = md.work[u];
            fuse_item<KMAX, WAVE, ROWS>(fp, md, sh, &md.items_big[it.x], it.y, lused, ok);
        } else if (u < nbig + nmed) {
            fuse_item<KMAX, WAVE, ROWS>(fp, md, sh, med_at(u - nbig), -1, lused, ok);
        } else if constexpr (WAVE) {
            fuse_item<KMAX, WAVE, ROWS>(fp, md, sh, small_at(u - nbig - nmed), -1, lused, ok);
        } else {
            const uint32_t k = (u - nbig - nmed) * nw + w;
            if (k < nsmall) fuse_wave_item<KMAX, WAVE, ROWS>(fp, md, sh, small_at(k), lused, ok);
            __syncthreads();
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) md.blk_stats[blk] = make_uint2(sh.uold, sh.unew);
    __syncthreads();
}

template <int KMAX, bool WAVE, bool ROWS>
__global__ __launch_bounds__(kLeafThreads, WAVE ? 1 : 3) void k_leaf_fuse(FrameParams fp, MapDev md)
{
    __shared__ LeafShared sh;
    leaf_fuse_range<KMAX, WAVE, ROWS>(fp, md, sh, blockIdx.x, gridDim.x);
}

// The maps mb.subset[0 .. nsubset) of a batch, all of this kernel's kind, each
// on its share of the grid.
template <int KMAX, bool WAVE, bool ROWS>
__global__ __launch_bounds__(kLeafThreads) void k_leaf_fuse_batch(MapBatch mb)
{
    __shared__ LeafShared sh;
    const int q = batch_map(mb.part_first, mb.nsubset, blockIdx.x), i = mb.subset[q];
    leaf_fuse_range<KMAX, WAVE, ROWS>(mb.fps[i], mb.mds[i], sh, blockIdx.x - mb.part_first[q],
                                      mb.part_first[q + 1] - mb.part_first[q]);
}


// ---------------------------------------------------------------------------
// 4'. per-leaf accumulation: geometry, or int32 labels with K <= 32 (Bayesian)
// ---------------------------------------------------------------------------
//
// Everything such a frame adds to a voxel is an integer: its observation count
// (W grows by it, Eq. (1)-(2)), its class counts (Eq. (6)) and its fixed-point
// distance sum.  Integer sums do not depend on the order of their terms, so a
// leaf's pairs are not sorted at all: each pair adds into its voxel's LDS
// accumulators with integer atomics (one set per frame of a multi-frame pass),
// then one lane per touched voxel applies them to the record, frame after
// frame.  The record is bitwise the same whatever order the pairs arrive in.

template <int KMAX, int FR>
struct AccShared {
    static constexpr int KW = KMAX > 0 ? (KMAX + 1) / 2 : 1;  // class counts as 16-bit fields, two to a word
    union {
        struct {  // one leaf per workgroup, indexed by voxel offset
            unsigned long long sum[FR][kLeafVoxels];
            uint32_t cnt[FR][kLeafVoxels];
            uint32_t lab[kLeafVoxels][KW];
        } b;
        struct {  // one leaf per wave, indexed by rank among the leaf's touched voxels
            unsigned long long sum[FR][kAccWavePairs];
            uint32_t cnt[FR][kAccWavePairs];
            uint32_t lab[kAccWavePairs][KW];
        } w[4];
    };
    uint32_t touch[4][kMaskWords];  // touched offsets of the workgroup's leaf, or of each wave's
    uint32_t pre[4][kMaskWords];    // touched offsets below each mask word (wave leaves)
    uint32_t item[4][32];           // the leaf item of the workgroup, or of each wave
    uint32_t uold, unew;
};

// Class counts of a voxel with more than 65535 observations in a unit (whose
// 16-bit counts may have wrapped), counted again from the unit's pairs, one
// class at a time, and added to its record.  Slow, and only for such voxels.
__device__ __noinline__ void acc_recount(const FrameParams &fp, const MapDev &md, long long rec, const uint2 *gkv,
                                         const int32_t *glab, uint32_t npairs, uint32_t o)
{
    float *R = md.vox + (size_t)rec * md.rec_stride;
    for (int k = 0; k < fp.K; ++k) {
        uint32_t c = 0;
        for (uint32_t t = 0; t < npairs; ++t) c += ((gkv[t].x >> kPidBits) == o && glab[t] == k) ? 1u : 0u;
        R[2 + k] += (float)c;
    }
}

// Applies one voxel's accumulators to its record: Eq. (1)-(2) frame after frame
// (each frame's run exactly as that frame alone), then Eq. (6).  sum and cnt
// point at frame 0's entry, the frames fstride apart; lab holds the 16-bit
// class counts.  A voxel with more than 65535 observations in the unit may have
// wrapped a 16-bit count: its labels are then counted again from the unit's
// pairs (gkv, glab, npairs), which only a workgroup unit passes.
template <int KMAX, int FR>
__device__ __forceinline__ void acc_apply(const FrameParams &fp, const MapDev &md, long long rec, bool existed,
                                          const unsigned long long *sum, const uint32_t *cnt, int fstride,
                                          const uint32_t *lab, int nf, const FixScale &fx, const uint2 *gkv,
                                          const int32_t *glab, uint32_t npairs, uint32_t o)
{
    constexpr int NV = (2 + KMAX + 3) / 4;
    const int nv = md.rec_stride / 4, K = fp.K;
    float4 *R = (float4 *)(md.vox + (size_t)rec * md.rec_stride);
    float r[4 * NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const float4 x = (existed && v < nv) ? R[v] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        r[4 * v + 0] = x.x;
        r[4 * v + 1] = x.y;
        r[4 * v + 2] = x.z;
        r[4 * v + 3] = x.w;
    }
    uint32_t ntot = 0;
#pragma unroll
    for (int f = 0; f < FR; ++f) {
        const uint32_t c = f < nf ? cnt[f * fstride] : 0u;
        if (c) {
            const float W0 = r[1], W1 = W0 + (float)c;
            r[0] = tsdf_mean(r[0], W0, W1, (long long)sum[f * fstride], fx.inv);
            r[1] = W1;
            ntot += c;
        }
    }
    const bool wrapped = ntot > 0xFFFFu;
    if constexpr (KMAX > 0) {
        if (!wrapped) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < K) r[2 + k] += (float)((lab[k >> 1] >> ((k & 1) << 4)) & 0xFFFFu);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
        if (v < nv) R[v] = make_float4(r[4 * v + 0], r[4 * v + 1], r[4 * v + 2], r[4 * v + 3]);
    if (KMAX > 0 && wrapped) acc_recount(fp, md, rec, gkv, glab, npairs, o);
}

// A leaf with more than kAccWavePairs pairs, whole, by one workgroup of
// kLeafThreads threads: its pairs stream through registers (kLeafBatch loads in
// flight per thread) into accumulators indexed by voxel offset.
template <int KMAX, int FR>
__device__ __forceinline__ void acc_block_unit(const FrameParams &fp, const MapDev &md, AccShared<KMAX, FR> &sh,
                                               const LeafItem *itp, unsigned long long lused, bool ok,
                                               const FixScale &fx, int nf)
{
    const int tid = threadIdx.x;
    if (tid < 32) sh.item[0][tid] = ((const uint32_t *)itp)[tid];
    {
        uint4 *p = (uint4 *)&sh.b;
        constexpr int nvec = (int)(sizeof(sh.b) / 16);
        for (int i = tid; i < nvec; i += blockDim.x) p[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    const uint32_t *it = sh.item[0];
    const uint32_t pos = it[0], n = it[1], bstart = it[2];
    const int islot = (int)it[3];
    const int slot = islot >= 0 ? islot : (int)(lused + (unsigned long long)(-1 - islot));
    // a new leaf's first insertion probe goes out with the pair loads
    const bool inserts = ok && islot < 0 && tid == 0;
    const unsigned long long lkey = ((unsigned long long)it[7] << 32) | it[6];
    uint32_t ih = 0;
    unsigned long long iprev = 0;
    if (inserts) iprev = map_insert_start(md, lkey, &ih);
    const uint2 *gkv = md.srt_kv + bstart;
    const int32_t *glab = md.srt_lab + bstart;
    for (uint32_t t0 = 0; t0 < n; t0 += kLeafBatch * blockDim.x) {
        uint32_t rk[kLeafBatch];
        float rv[kLeafBatch];
        int32_t rl[kLeafBatch];
#pragma unroll
        for (int u = 0; u < kLeafBatch; ++u) {
            const uint32_t t = t0 + u * blockDim.x + tid;
            const uint2 e = t < n ? gkv[t] : make_uint2(0u, 0u);
            rk[u] = e.x;
            rv[u] = __uint_as_float(e.y);
            rl[u] = (KMAX > 0 && t < n) ? glab[t] : 0;
        }
#pragma unroll
        for (int u = 0; u < kLeafBatch; ++u)
            if (t0 + u * blockDim.x + tid < n) {
                const uint32_t o = rk[u] >> kPidBits;
                const int f = FR > 1 ? pass_frame(fp, rk[u] & kPidMask) : 0;
                atomicAdd(&sh.b.cnt[f][o], 1u);
                atomicAdd(&sh.b.sum[f][o], (unsigned long long)fix_q(rv[u], fx.s));
                if constexpr (KMAX > 0) atomicAdd(&sh.b.lab[o][rl[u] >> 1], 1u << ((rl[u] & 1) << 4));
            }
    }
    __syncthreads();
    {
        // touched offsets: wave w covers offsets 64 w + [0, 64) and 256 + 64 w + [0, 64)
        uint32_t c0 = 0, c1 = 0;
#pragma unroll
        for (int f = 0; f < FR; ++f)
            if (f < nf) {
                c0 += sh.b.cnt[f][tid];
                c1 += sh.b.cnt[f][tid + 256];
            }
        const unsigned long long b0 = __ballot(c0 != 0u), b1 = __ballot(c1 != 0u);
        const int w = tid >> 6;
        if (lane_id() == 0) {
            sh.touch[0][2 * w] = (uint32_t)b0;
            sh.touch[0][2 * w + 1] = (uint32_t)(b0 >> 32);
            sh.touch[0][8 + 2 * w] = (uint32_t)b1;
            sh.touch[0][9 + 2 * w] = (uint32_t)(b1 >> 32);
        }
    }
    __syncthreads();
    // thread t takes the touched offsets of rank t, t + blockDim.x, ...
    uint32_t ntouch = 0;
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) ntouch += __popc(sh.touch[0][w]);
    if (ok) {
        for (uint32_t r = tid; r < ntouch; r += blockDim.x) {
            uint32_t w = 0, before = 0, bits = 0;
            for (; w < (uint32_t)kMaskWords; ++w) {
                bits = sh.touch[0][w];
                const uint32_t c = __popc(bits);
                if (r < before + c) break;
                before += c;
            }
            const uint32_t o = (w << 5) + select_bit(bits, r - before);
            const long long rec = (long long)(int)it[8 + (o >> 6)] * kPageVoxels + (o & (kPageVoxels - 1));
            const bool existed = (it[16 + (o >> 5)] >> (o & 31)) & 1u;
            acc_apply<KMAX, FR>(fp, md, rec, existed, &sh.b.sum[0][o], &sh.b.cnt[0][o], kLeafVoxels, sh.b.lab[o], nf,
                                fx, gkv, glab, n, o);
        }
    }
    if (tid == 0) {
        uint32_t uo = 0, un = 0;
        for (int w = 0; w < kMaskWords; ++w) {
            uo += __popc(sh.touch[0][w] & it[16 + w]);
            un += __popc(sh.touch[0][w] & ~it[16 + w]);
        }
        sh.uold += uo;
        sh.unew += un;
    }
    // leaf bookkeeping: the unit owns the whole leaf
    if (ok) {
        if (inserts) {
            map_insert_finish(md, lkey, slot, ih, iprev);
            md.leaf_key[slot] = lkey;
        }
        if (tid < kLeafPages) md.leaf_page[(size_t)slot * kLeafPages + tid] = (int)it[8 + tid];
        if (tid < kMaskWords) md.leaf_occ[(size_t)slot * kMaskWords + tid] = it[16 + tid] | sh.touch[0][tid];
    }
    if (tid == 0) {
        md.skeys[pos] = kEmptyKey;
        md.pos_count[pos] = 0u;
        md.pos_slab[pos] = 0u;
    }
    __syncthreads();
}

// A leaf with at most kAccWavePairs pairs, by one wave (two pairs per lane):
// accumulators indexed by the rank of the voxel among the leaf's touched
// voxels.  Waves run such leaves independently, four per workgroup.
template <int KMAX, int FR>
__device__ __forceinline__ void acc_wave_unit(const FrameParams &fp, const MapDev &md, AccShared<KMAX, FR> &sh,
                                              const LeafItem *itp, unsigned long long lused, bool ok,
                                              const FixScale &fx, int nf)
{
    const int lane = lane_id(), w = threadIdx.x >> 6;
    auto &A = sh.w[w];
    uint32_t *wi = sh.item[w], *wt = sh.touch[w], *wp = sh.pre[w];
    if (lane < 32) wi[lane] = ((const uint32_t *)itp)[lane];
    if (lane < kMaskWords) wt[lane] = 0u;
    {
        uint4 *p = (uint4 *)&A;
        constexpr int nvec = (int)(sizeof(A) / 16);
        for (int i = lane; i < nvec; i += 64) p[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    wave_sync();
    const uint32_t pos = wi[0], n = wi[1], bstart = wi[2];
    const int islot = (int)wi[3];
    const int slot = islot >= 0 ? islot : (int)(lused + (unsigned long long)(-1 - islot));
    const bool inserts = ok && islot < 0 && lane == 0;
    const unsigned long long lkey = ((unsigned long long)wi[7] << 32) | wi[6];
    uint32_t ih = 0;
    unsigned long long iprev = 0;
    if (inserts) iprev = map_insert_start(md, lkey, &ih);
    uint32_t kq[2];
    float vq[2];
    int32_t lq[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const uint32_t i = lane + 64 * q;
        const bool has = i < n;
        const uint2 e = has ? md.srt_kv[bstart + i] : make_uint2(0u, 0u);
        kq[q] = e.x;
        vq[q] = __uint_as_float(e.y);
        lq[q] = (KMAX > 0 && has) ? md.srt_lab[bstart + i] : 0;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
        if (lane + 64 * q < n) {
            const uint32_t o = kq[q] >> kPidBits;
            atomicOr(&wt[o >> 5], 1u << (o & 31));
        }
    wave_sync();
    // rank of a touched offset: the touched offsets below its mask word, plus
    // those below it in the word
    const uint32_t pc = lane < kMaskWords ? (uint32_t)__popc(wt[lane]) : 0u;
    const uint32_t incl = wave_incl_scan(pc);
    if (lane < kMaskWords) wp[lane] = incl - pc;
    const uint32_t nvox = (uint32_t)__shfl((int)incl, kMaskWords - 1, 64);
    wave_sync();
#pragma unroll
    for (int q = 0; q < 2; ++q)
        if (lane + 64 * q < n) {
            const uint32_t o = kq[q] >> kPidBits;
            const uint32_t ci = wp[o >> 5] + (uint32_t)__popc(wt[o >> 5] & ((1u << (o & 31)) - 1u));
            const int f = FR > 1 ? pass_frame(fp, kq[q] & kPidMask) : 0;
            atomicAdd(&A.cnt[f][ci], 1u);
            atomicAdd(&A.sum[f][ci], (unsigned long long)fix_q(vq[q], fx.s));
            if constexpr (KMAX > 0) atomicAdd(&A.lab[ci][lq[q] >> 1], 1u << ((lq[q] & 1) << 4));
        }
    wave_sync();
    if (ok) {
        for (uint32_t ci = lane; ci < nvox; ci += 64) {
            // offset of rank ci: its mask word, then its bit there
            uint32_t wd = 0;
            while (wd + 1 < (uint32_t)kMaskWords && wp[wd + 1] <= ci) ++wd;
            const uint32_t o = (wd << 5) + select_bit(wt[wd], ci - wp[wd]);
            const long long rec = (long long)(int)wi[8 + (o >> 6)] * kPageVoxels + (o & (kPageVoxels - 1));
            const bool existed = (wi[16 + (o >> 5)] >> (o & 31)) & 1u;
            acc_apply<KMAX, FR>(fp, md, rec, existed, &A.sum[0][ci], &A.cnt[0][ci], kAccWavePairs, A.lab[ci], nf, fx,
                                nullptr, nullptr, 0u, o);
        }
    }
    // statistics and leaf bookkeeping
    const uint32_t tw = lane < kMaskWords ? wt[lane] : 0u;
    const uint32_t occ = lane < kMaskWords ? wi[16 + lane] : 0u;
    uint32_t uo = __popc(tw & occ), un = __popc(tw & ~occ);
    for (int d = 32; d > 0; d >>= 1) {
        uo += __shfl_xor(uo, d, 64);
        un += __shfl_xor(un, d, 64);
    }
    if (lane == 0) {
        atomicAdd(&sh.uold, uo);
        atomicAdd(&sh.unew, un);
    }
    if (ok) {
        if (inserts) {
            map_insert_finish(md, lkey, slot, ih, iprev);
            md.leaf_key[slot] = lkey;
        }
        if (lane < kLeafPages) md.leaf_page[(size_t)slot * kLeafPages + lane] = (int)wi[8 + lane];
        if (lane < kMaskWords) md.leaf_occ[(size_t)slot * kMaskWords + lane] = occ | tw;
    }
    if (lane == 0) {
        md.skeys[pos] = kEmptyKey;
        md.pos_count[pos] = 0u;
        md.pos_slab[pos] = 0u;
    }
    wave_sync();
}

// The accumulation kernel's work of one map's frame for blocks blk, blk + nblk,
// ...: the leaves done by a workgroup (the larger ones first), then groups of
// four small leaves, one per wave.  Block statistics go to md.blk_stats[blk].
template <int KMAX, int FR>
__device__ __forceinline__ void leaf_acc_range(const FrameParams &fp, const MapDev &md, AccShared<KMAX, FR> &sh,
                                               uint32_t blk, uint32_t nblk)
{
    const DevState *st = md.st;
    const unsigned long long lused = st->leaves_used;
    const bool ok = md.fs->frame_err.v == 0 && st->pass_failed == 0 &&
                    lused + md.fs->new_leaves.v <= (unsigned long long)md.max_leaves &&
                    st->pages_used + md.fs->new_pages.v <= (unsigned long long)md.max_pages;
    if (threadIdx.x == 0) {
        sh.uold = 0;
        sh.unew = 0;
    }
    __syncthreads();
    const uint32_t medf = (uint32_t)md.fs->n_lists, smallf = (uint32_t)(md.fs->n_lists >> 32);
    const uint32_t nmed = medf + (uint32_t)md.fs->n_lists_tail;
    const uint32_t nsmall = smallf + (uint32_t)(md.fs->n_lists_tail >> 32);
    const uint32_t last = md.hmask;
    const uint32_t nw = blockDim.x >> 6, w = threadIdx.x >> 6;
    const uint32_t nunits = nmed + (nsmall + nw - 1) / nw;
    const FixScale fx = fix_scale(fp);
    const int nf = fp.nsub > 1 ? fp.nsub : 1;
    for (uint32_t u = blk; u < nunits; u += nblk) {
        if (u < nmed) {
            acc_block_unit<KMAX, FR>(fp, md, sh, &md.items[u < medf ? u : last - (u - medf)], lused, ok, fx, nf);
        } else {
            const uint32_t k = (u - nmed) * nw + w;
            if (k < nsmall)
                acc_wave_unit<KMAX, FR>(fp, md, sh, &md.items_small[k < smallf ? k : last - (k - smallf)], lused, ok,
                                        fx, nf);
            __syncthreads();
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) md.blk_stats[blk] = make_uint2(sh.uold, sh.unew);
    __syncthreads();
}

template <int KMAX, int FR>
__global__ __launch_bounds__(kLeafThreads, 3) void k_leaf_acc(FrameParams fp, MapDev md)
{
    __shared__ AccShared<KMAX, FR> sh;
    leaf_acc_range<KMAX, FR>(fp, md, sh, blockIdx.x, gridDim.x);
}

// The maps mb.subset[0 .. nsubset) of a batch (one frame each), all of this
// kernel's kind, each on its share of the grid.
template <int KMAX>
__global__ __launch_bounds__(kLeafThreads, 3) void k_leaf_acc_batch(MapBatch mb)
{
    __shared__ AccShared<KMAX, 1> sh;
    const int q = batch_map(mb.part_first, mb.nsubset, blockIdx.x), i = mb.subset[q];
    leaf_acc_range<KMAX, 1>(mb.fps[i], mb.mds[i], sh, blockIdx.x - mb.part_first[q],
                            mb.part_first[q + 1] - mb.part_first[q]);
}

// One wave per voxel descriptor of the frame (open set, wide class counts,
// most-recent open set): the combine of the wave-per-voxel leaf kernels, run
// over all voxels of the frame at once so that the heavy voxels spread over the
// whole GPU.  Consecutive descriptors (neighbouring voxels, which share
// observations) go to workgroups on the same XCD.
template <int KMAX>
__device__ __forceinline__ void voxel_combine_range(const FrameParams &fp, const MapDev &md, uint32_t blk,
                                                    uint32_t nblk)
{
    const uint32_t nv = md.fs->n_vox.v;
    const uint32_t nw = blockDim.x >> 6, w = threadIdx.x >> 6;
    // blocks are dealt to the 8 XCDs round robin: give each XCD a contiguous
    // share (XCD r holds the nblk / 8 blocks, plus one if r < nblk % 8, whose
    // index is r modulo 8; a one-to-one map of [0, nblk) for any nblk)
    const uint32_t r = blk % 8, q = nblk / 8, m = nblk % 8;
    const uint32_t vb = r * q + min(r, m) + blk / 8;
    const uint32_t step = nblk * nw;
    if constexpr (KMAX >= 8) {
        // L >= 512: a wave's voxels one after another, each one's descriptor requested
        // two voxels ahead and its observations' point indices and distances
        // one voxel ahead, so that only the rows and the record are waited
        // for (indices past the end read the wave's first voxel again)
        const uint32_t lane = (uint32_t)lane_id();
        const uint32_t v0 = vb * nw + w;
        if (v0 >= nv) return;
        uint4 d = md.vox_list[v0];
        uint32_t kl = lane < (d.y & 0x7FFFFFFFu) ? md.pair_key[d.z + lane] & kPidMask : 0u;
        float vl = lane < (d.y & 0x7FFFFFFFu) ? md.pair_tsdf[d.z + lane] : 0.0f;
        uint32_t vn = v0 + step;
        uint4 dn = md.vox_list[vn < nv ? vn : v0];
        for (;;) {
            const bool more = vn < nv;
            const uint32_t nn = more ? dn.y & 0x7FFFFFFFu : 0u;
            const uint32_t kn = lane < nn ? md.pair_key[dn.z + lane] & kPidMask : 0u;
            const float vln = lane < nn ? md.pair_tsdf[dn.z + lane] : 0.0f;
            const uint32_t vnn = vn + step;
            const uint4 dnn = md.vox_list[vnn < nv ? vnn : v0];
            combine_wave_vec<(KMAX > 0 ? KMAX : 1)>(fp, md, md.pair_key + d.z, md.pair_tsdf + d.z,
                                                    d.y & 0x7FFFFFFFu, (long long)d.x, (d.y >> 31) != 0u, kl, vl);
            if (!more) break;
            d = dn;
            kl = kn;
            vl = vln;
            vn = vnn;
            dn = dnn;
        }
    } else {
        // the other kinds one voxel at a time: for L <= 256 (few observations
        // per voxel) requesting ahead gains nothing and costs the registers
        // of more waves
        for (uint32_t v = vb * nw + w; v < nv; v += step) {
            const uint4 d = md.vox_list[v];
            const uint32_t n = d.y & 0x7FFFFFFFu;
            const bool existed = (d.y >> 31) != 0u;
            const uint32_t *keys = md.pair_key + d.z;
            const float *vals = md.pair_tsdf + d.z;
            if constexpr (KMAX > 0)
                combine_wave_vec<(KMAX > 0 ? KMAX : 1)>(fp, md, keys, vals, n, (long long)d.x, existed);
            else if constexpr (KMAX < 0)
                combine_last_wave(fp, md, keys, vals, n, (long long)d.x, existed);
            else
                combine_wave(fp, md, keys, vals, n, (long long)d.x, existed);
        }
    }
}

// The wave combine of the maps mb.subset[0 .. nsubset) of a batch in one
// launch: their voxel lists are taken as one list, map after map, and the
// whole grid strides over it as voxel_combine_range does over one map's, so
// that the work spreads evenly whatever the maps' sizes.
constexpr int kMaxBatchMaps = 1024;
template <int KMAX>
__device__ __forceinline__ void voxel_combine_maps(const MapBatch &mb, uint32_t blk, uint32_t nblk)
{
    __shared__ uint32_t pre[kMaxBatchMaps + 1];  // first voxel of each map in the joint list, then the total
    __shared__ uint32_t wsum[4];
    const int ns = min(mb.nsubset, kMaxBatchMaps), tid = threadIdx.x;
    uint32_t c[4], t = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int q = tid * 4 + u;
        c[u] = q < ns ? mb.mds[mb.subset[q]].fs->n_vox.v : 0u;
        t += c[u];
    }
    const uint32_t incl = wave_incl_scan(t);
    if (lane_id() == 63) wsum[tid >> 6] = incl;
    __syncthreads();
    uint32_t run = incl - t;
    for (int w = 0; w < (tid >> 6); ++w) run += wsum[w];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int q = tid * 4 + u;
        if (q < ns) pre[q] = run;
        run += c[u];
    }
    if (tid == 0) pre[ns] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    const uint32_t nv = pre[ns];
    const uint32_t nw = blockDim.x >> 6, w = tid >> 6;
    // the XCD deal of voxel_combine_range
    const uint32_t r = blk % 8, qb = nblk / 8, m = nblk % 8;
    const uint32_t vb = r * qb + min(r, m) + blk / 8;
    const uint32_t step = nblk * nw;
    int q = 0;
    for (uint32_t v = vb * nw + w; v < nv; v += step) {
        while (pre[q + 1] <= v) ++q;  // the map of joint voxel v (pre[ns] = nv > v)
        const int i = mb.subset[q];
        const MapDev &md = mb.mds[i];
        const FrameParams &fp = mb.fps[i];
        const uint4 d = md.vox_list[v - pre[q]];
        const uint32_t n = d.y & 0x7FFFFFFFu;
        const bool existed = (d.y >> 31) != 0u;
        const uint32_t *keys = md.pair_key + d.z;
        const float *vals = md.pair_tsdf + d.z;
        if constexpr (KMAX > 0)
            combine_wave_vec<(KMAX > 0 ? KMAX : 1)>(fp, md, keys, vals, n, (long long)d.x, existed);
        else if constexpr (KMAX < 0)
            combine_last_wave(fp, md, keys, vals, n, (long long)d.x, existed);
        else
            combine_wave(fp, md, keys, vals, n, (long long)d.x, existed);
    }
}

// Workgroups per CU the combine kernels are built for: the vectorised kinds are
// bound by the latency of their row and record accesses, so they keep enough
// waves in flight (register budgets 72, 100, 72, 168 for L = 64, 128, 256, 512).
__host__ __device__ constexpr int combine_min_blocks(int kmax)
{
    return kmax == 1 ? 7 : (kmax == 2 ? 5 : (kmax == 4 ? 7 : (kmax == 8 ? 3 : 1)));
}

template <int KMAX>
__global__ __launch_bounds__(256, combine_min_blocks(KMAX)) void k_voxel_combine(FrameParams fp, MapDev md)
{
    voxel_combine_range<KMAX>(fp, md, blockIdx.x, gridDim.x);
}

template <int KMAX>
__global__ __launch_bounds__(256, combine_min_blocks(KMAX)) void k_voxel_combine_batch(MapBatch mb)
{
    voxel_combine_maps<KMAX>(mb, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// 5. commit (one workgroup)
// ---------------------------------------------------------------------------

struct CommitShared {
    unsigned long long s_old[256], s_new[256];
};

__device__ __forceinline__ void frame_commit_block(const FrameParams &fp, const MapDev &md, CommitShared &cs)
{
    unsigned long long *s_old = cs.s_old, *s_new = cs.s_new;
    DevState *st = md.st;
    // the frame's counters and the map's state are read together with the
    // per-block statistics (one round trip for all of them)
    unsigned long long nl = 0, np = 0, lu = 0, pu = 0, vu = 0;
    uint32_t ferr = 0, nrej = 0, npairs = 0, ntouch = 0;
    int failed = 0, status = 0;
    if (threadIdx.x == 0) {
        nl = md.fs->new_leaves.v;
        np = md.fs->new_pages.v;
        ferr = md.fs->frame_err.v;
        nrej = md.fs->rejected.v;
        npairs = md.fs->pairs.v;
        ntouch = md.fs->n_touched.v;
        failed = st->pass_failed;
        status = st->status;
        lu = st->leaves_used;
        pu = st->pages_used;
        vu = st->voxels_used;
    }
    unsigned long long uo = 0, un = 0;
    for (int b0 = threadIdx.x; b0 < md.leaf_blocks; b0 += 8 * blockDim.x) {
        uint2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int b = b0 + q * blockDim.x;
            v[q] = b < md.leaf_blocks ? md.blk_stats[b] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            uo += v[q].x;
            un += v[q].y;
        }
    }
    s_old[threadIdx.x] = uo;
    s_new[threadIdx.x] = un;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < (unsigned)d) {
            s_old[threadIdx.x] += s_old[threadIdx.x + d];
            s_new[threadIdx.x] += s_new[threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // after a multi-frame pass that could not be applied, the frames that
        // follow it in the same sequence call are skipped too: the host
        // integrates them again one by one
        const bool skipped = failed != 0;
        const bool ok = !skipped && ferr == 0 && lu + nl <= (unsigned long long)md.max_leaves &&
                        pu + np <= (unsigned long long)md.max_pages;
        if (ok) {
            st->leaves_used = lu + nl;
            st->pages_used = pu + np;
            st->voxels_used = vu + s_new[0];
        } else if (!skipped && fp.nsub > 1) {
            st->pass_failed = 1 + fp.pass_first;
        } else if (!skipped && status == SLIM_OK) {
            st->status = SLIM_ERR_CAPACITY;
        }
        if (!skipped && (ok || fp.nsub <= 1)) {
            st->last_points = fp.n;
            st->last_rejected = nrej;
            st->last_pairs = npairs;
            st->last_touched = ntouch;
            st->last_new_leaves = nl;
            st->last_u_old = (long long)s_old[0];
            st->last_u_new = (long long)s_new[0];
            st->last_status = ok ? SLIM_OK : SLIM_ERR_CAPACITY;
        }
        md.fs->n_touched.v = 0;
        md.fs->pairs.v = 0;
        md.fs->rejected.v = 0;
        md.fs->new_leaves.v = 0;
        md.fs->new_pages.v = 0;
        md.fs->pair_cursor.v = 0;
        md.fs->work_big.v = 0;
        md.fs->n_lists = 0;
        md.fs->n_lists_tail = 0;
        md.fs->n_vox.v = 0;
        md.fs->frame_err.v = 0;
    }
}

__global__ __launch_bounds__(256) void k_frame_commit(FrameParams fp, MapDev md)
{
    __shared__ CommitShared cs;
    frame_commit_block(fp, md, cs);
}

__global__ __launch_bounds__(256) void k_frame_commit_batch(MapBatch mb)
{
    __shared__ CommitShared cs;
    frame_commit_block(mb.fps[blockIdx.x], mb.mds[blockIdx.x], cs);
}

// ---------------------------------------------------------------------------
// 6. the persistent batched launch
// ---------------------------------------------------------------------------
//
// One launch integrates one frame into each of many maps.  Its workgroups stay
// resident and take work items from an integer queue in order: the ray-chunk
// items of every map's walk, then every map's planning, bucketing, leaf-tile,
// voxel-combine and commit items.  An item of a stage starts once all items of
// the previous stage of the same map have finished (a per-map, per-stage
// counter), so the stages of different maps overlap and a large frame does
// not hold up a small one.  Items are taken in queue order and an item only
// waits for items earlier in the queue, which are held by running workgroups:
// the queue always drains, whatever the number of workgroups.  Every item runs
// the same code as the per-stage kernels, so the maps are bitwise the same as
// after the per-stage launches (and the per-map calls).

// Leaf-kernel variants whose voxels are combined by k_voxel_combine (one wave
// per voxel), with that kernel's template argument; -2: combined in the leaf kernel.
__host__ __device__ int voxel_combine_arg(int kind)
{
    switch (kind) {
    case 8: return 0;
    case 10: return -1;
    case 11: return 1;
    case 12: return 2;
    case 13: return 4;
    case 14: return 8;
    case 15: return 16;
    default: return -2;
    }
}

static_assert(kWalkThreads == 256 && kLeafThreads == 256, "persistent items assume 256-thread workgroups");

union PersistShared {
    WalkShared walk;
    LeafShared leaf;
    AccShared<0, 1> acc0;
    AccShared<8, 1> acc8;
    AccShared<16, 1> acc16;
    AccShared<24, 1> acc24;
    AccShared<32, 1> acc32;
    CommitShared commit;
};
// The launch's LDS, one copy per workgroup, named directly by the stage
// functions below (a reference passed to a called function would lose its
// address space).
static __shared__ PersistShared g_ps;

template <int KMAX>
__device__ __forceinline__ AccShared<KMAX, 1> &persist_acc_lds()
{
    if constexpr (KMAX == 0) return g_ps.acc0;
    else if constexpr (KMAX == 8) return g_ps.acc8;
    else if constexpr (KMAX == 16) return g_ps.acc16;
    else if constexpr (KMAX == 24) return g_ps.acc24;
    else return g_ps.acc32;
}

// A waiting workgroup gives up after this many polls (seconds), raises the
// launch's abort flag and marks its map failed: every later item is then
// skipped, so the launch always ends.  The queue order makes this unreachable
// in a correct launch; it is a guard against a broken item list.
constexpr uint32_t kPersistSpinLimit = 1u << 22;

// Arguments of a called stage function arrive in vector registers; the
// workgroup's item is the same in every lane, so they are taken back as
// wave-uniform values on entry.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

template <class T>
__device__ __forceinline__ const T &uni_ref(const T &r)
{
    const unsigned long long p = (unsigned long long)&r;
    return *(const T *)(((unsigned long long)uni((uint32_t)(p >> 32)) << 32) | uni((uint32_t)p));
}

// Each stage variant is a function of its own (called, not inlined), so it is
// register-allocated alone, as in its own kernel.
__device__ __noinline__ void persist_walk(const FrameParams &fpa, const MapDev &mda, uint32_t b0a, uint32_t nba)
{
    const FrameParams &fp = uni_ref(fpa);
    const MapDev &md = uni_ref(mda);
    const uint32_t b0 = uni(b0a), b1 = b0 + uni(nba);
    for (uint32_t b = b0; b < b1; ++b) {
        walk_emit_block(fp, md, (int)b, g_ps.walk);
        __syncthreads();
    }
}

__device__ __noinline__ void persist_plan(const FrameParams &fp, const MapDev &md, uint32_t j, uint32_t cnt)
{
    leaf_plan_range(uni_ref(fp), uni_ref(md), uni(j), uni(cnt));
}

__device__ __noinline__ void persist_bucket(const FrameParams &fp, const MapDev &md, uint32_t j, uint32_t cnt)
{
    pair_bucket_range(uni_ref(fp), uni_ref(md), uni(j), uni(cnt));
}

template <int KMAX>
__device__ __noinline__ void persist_acc(const FrameParams &fp, const MapDev &md, uint32_t j, uint32_t cnt)
{
    leaf_acc_range<KMAX, 1>(uni_ref(fp), uni_ref(md), persist_acc_lds<KMAX>(), uni(j), uni(cnt));
}

template <int KMAX, bool WAVE, bool ROWS>
__device__ __noinline__ void persist_fuse(const FrameParams &fp, const MapDev &md, uint32_t j, uint32_t cnt)
{
    leaf_fuse_range<KMAX, WAVE, ROWS>(uni_ref(fp), uni_ref(md), g_ps.leaf, uni(j), uni(cnt));
}

template <int KMAX>
__device__ __noinline__ void persist_comb(const FrameParams &fp, const MapDev &md, uint32_t j, uint32_t cnt)
{
    voxel_combine_range<KMAX>(uni_ref(fp), uni_ref(md), uni(j), uni(cnt));
}

__device__ __noinline__ void persist_commit(const FrameParams &fp, const MapDev &md)
{
    frame_commit_block(uni_ref(fp), uni_ref(md), g_ps.commit);
}

__device__ __forceinline__ void persist_leaf(int kind, const FrameParams &fp, const MapDev &md, uint32_t j,
                                             uint32_t cnt)
{
    switch (kind) {
    case 0: persist_acc<0>(fp, md, j, cnt); break;
    case 1: persist_acc<8>(fp, md, j, cnt); break;
    case 2: persist_acc<16>(fp, md, j, cnt); break;
    case 3: persist_acc<24>(fp, md, j, cnt); break;
    case 4: persist_acc<32>(fp, md, j, cnt); break;
    case 5: persist_fuse<8, false, true>(fp, md, j, cnt); break;
    case 6: persist_fuse<16, false, true>(fp, md, j, cnt); break;
    case 7: persist_fuse<32, false, true>(fp, md, j, cnt); break;
    case 16: persist_fuse<24, false, true>(fp, md, j, cnt); break;
    case 9: persist_fuse<-1, false, false>(fp, md, j, cnt); break;
    case 10: persist_fuse<-1, true, false>(fp, md, j, cnt); break;
    case 11: persist_fuse<1, true, false>(fp, md, j, cnt); break;
    case 12: persist_fuse<2, true, false>(fp, md, j, cnt); break;
    case 13: persist_fuse<4, true, false>(fp, md, j, cnt); break;
    case 14: persist_fuse<8, true, false>(fp, md, j, cnt); break;
    case 15: persist_fuse<16, true, false>(fp, md, j, cnt); break;
    default: persist_fuse<0, true, false>(fp, md, j, cnt); break;
    }
}

__device__ __forceinline__ void persist_combine(int kind, const FrameParams &fp, const MapDev &md, uint32_t j,
                                                uint32_t cnt)
{
    switch (voxel_combine_arg(kind)) {
    case 0: persist_comb<0>(fp, md, j, cnt); break;
    case -1: persist_comb<-1>(fp, md, j, cnt); break;
    case 1: persist_comb<1>(fp, md, j, cnt); break;
    case 2: persist_comb<2>(fp, md, j, cnt); break;
    case 4: persist_comb<4>(fp, md, j, cnt); break;
    case 8: persist_comb<8>(fp, md, j, cnt); break;
    case 16: persist_comb<16>(fp, md, j, cnt); break;
    default: break;
    }
}

__global__ __launch_bounds__(256, 3) void k_batch_persistent(PersistArgs a)
{
    __shared__ uint4 s_item;
    __shared__ uint32_t s_skip;
    // Thread 0 alone talks to the queue, in one place per round: it counts the
    // item the workgroup has just finished (after the release below), takes
    // the next one and waits for its dependency.  Keeping that one guarded
    // region per round, and the item wave-uniform, keeps every barrier of the
    // loop in uniform control flow.
    uint32_t finished = kPersistEnd;  // counter of the item the workgroup finished last
    for (;;) {
        if (threadIdx.x == 0) {
            if (finished != kPersistEnd) atomicAdd(&a.ctl[kPersistCtlDone + finished], 1u);
            const uint32_t it = atomicAdd(&a.ctl[0], 1u);
            uint4 item = make_uint4(kPersistEnd, 0u, 0u, 0u);
            uint32_t skip = 0;
            if (it < a.nitems) {
                item = a.items[it];
                if (item.w != kPersistNoDep) {
                    // wait for every item of the map's previous stage
                    const uint32_t *done = &a.ctl[kPersistCtlDone + (item.w & 0xFFFFu)];
                    const uint32_t need = item.w >> 16;
                    uint32_t polls = 0;
                    while (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (++polls > kPersistSpinLimit) {
                            atomicOr(&a.ctl[kPersistCtlAbort], 1u);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
                skip = __hip_atomic_load(&a.ctl[kPersistCtlAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __threadfence();
                // after an abort the map's remaining items are skipped and the map is marked failed
                const DevState *st = a.mds[item.x & 0xFFFFu].st;
                if (skip && st->status == SLIM_OK) ((DevState *)st)->status = SLIM_ERR_DEVICE;
            }
            s_item = item;
            s_skip = skip;
        }
        __syncthreads();
        // every thread reads the same item: taken as wave-uniform values, so
        // the loop and its exit stay uniform
        const uint4 item = make_uint4(__builtin_amdgcn_readfirstlane(s_item.x), __builtin_amdgcn_readfirstlane(s_item.y),
                                      __builtin_amdgcn_readfirstlane(s_item.z), __builtin_amdgcn_readfirstlane(s_item.w));
        const uint32_t skip = __builtin_amdgcn_readfirstlane(s_skip);
        if (item.x == kPersistEnd) break;
        // acquire (every wave): what the previous stage wrote on other XCDs is visible
        __threadfence();
        const uint32_t i = item.x & 0xFFFFu, stage = (item.x >> 16) & 0xFFu;
        const int kind = (int)(item.x >> 24);
        const FrameParams &fp = a.fps[i];
        const MapDev &md = a.mds[i];
        if (!skip) {
            switch (stage) {
            case 0: persist_walk(fp, md, item.y, item.z); break;
            case 1: persist_plan(fp, md, item.y, item.z); break;
            case 2: persist_bucket(fp, md, item.y, item.z); break;
            case 3: persist_leaf(kind, fp, md, item.y, item.z); break;
            case 4: persist_combine(kind, fp, md, item.y, item.z); break;
            default: persist_commit(fp, md); break;
            }
        }
        // release: this item's writes reach the device level before thread 0
        // counts it, at the top of the next round
        __threadfence();
        __syncthreads();
        finished = i * kPersistStages + stage;
    }
}

int persistent_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_persistent, 256, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_integrate_persistent(const PersistArgs &a, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_persistent, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// Variant of the leaf kernel a frame needs: 0 geometry; 1..4 labels with
// 8/16/24/32 classes in registers; 5..7 probability or logit rows with 8/16/32 (17..24 classes: 16);
// 8 one wave per voxel (open set, or more than 32 classes); 9 and 10 the
// most-recent-measurement modes (closed: lane per voxel; open: wave per voxel);
// 11..15 the open set with L = 64, 128, 256, 512, 1024 read as whole words;
// 16 probability or logit rows with 24 classes in registers.
int leaf_kernel_kind(const FrameParams &fp)
{
    if (fp.last) return fp.L > 0 ? 10 : 9;
    if (fp.L > 0 && (fp.L & 63) == 0 && ((uintptr_t)fp.sem & 15u) == 0) {
        // embeddings whose rows split into whole 4- to 16-byte words per lane
        const int v = fp.L >> 6;
        const bool bf = fp.sem_kind == SLIM_IN_EMB_BF16;
        if (v == 1 && !bf) return 11;
        if (v == 2) return 12;
        if (v == 4) return 13;
        if (v == 8) return 14;
        if (v == 16) return 15;
    }
    if (fp.L > 0 || fp.K > 32) return 8;
    if (fp.K == 0) return 0;
    const bool rows = fp.sem_kind == SLIM_IN_PROB_F32 || fp.sem_kind == SLIM_IN_LOGIT_F32;
    if (rows) return fp.K > 24 ? 7 : (fp.K > 16 ? 16 : (fp.K > 8 ? 6 : 5));
    return fp.K > 24 ? 4 : (fp.K > 16 ? 3 : (fp.K > 8 ? 2 : 1));
}

// Grid of the wave combine.  Its blocks take equal static shares of the
// voxels, so the kinds built for 3 or 7 workgroups per CU (L = 512, 256 as
// whole words) run two rounds of what the CUs hold at once, the others the leaf
// kernel's grid.
int combine_blocks(int kind, const LaunchShape &shape)
{
    const int k = voxel_combine_arg(kind);
    return (k == 4 || k == 8) ? 2 * combine_min_blocks(k) * shape.cus : shape.leaf_blocks;
}

static void launch_voxel_combine(int kind, const FrameParams &fp, const MapDev &md, int blocks, hipStream_t s)
{
    const dim3 gl(blocks), bl(256);
    switch (voxel_combine_arg(kind)) {
    case 0: hipLaunchKernelGGL((k_voxel_combine<0>), gl, bl, 0, s, fp, md); break;
    case -1: hipLaunchKernelGGL((k_voxel_combine<-1>), gl, bl, 0, s, fp, md); break;
    case 1: hipLaunchKernelGGL((k_voxel_combine<1>), gl, bl, 0, s, fp, md); break;
    case 2: hipLaunchKernelGGL((k_voxel_combine<2>), gl, bl, 0, s, fp, md); break;
    case 4: hipLaunchKernelGGL((k_voxel_combine<4>), gl, bl, 0, s, fp, md); break;
    case 8: hipLaunchKernelGGL((k_voxel_combine<8>), gl, bl, 0, s, fp, md); break;
    case 16: hipLaunchKernelGGL((k_voxel_combine<16>), gl, bl, 0, s, fp, md); break;
    default: break;
    }
}

static void launch_voxel_combine_batch(int kind, const MapBatch &mb, int blocks, hipStream_t s)
{
    const dim3 gl(blocks), bl(256);
    switch (voxel_combine_arg(kind)) {
    case 0: hipLaunchKernelGGL((k_voxel_combine_batch<0>), gl, bl, 0, s, mb); break;
    case -1: hipLaunchKernelGGL((k_voxel_combine_batch<-1>), gl, bl, 0, s, mb); break;
    case 1: hipLaunchKernelGGL((k_voxel_combine_batch<1>), gl, bl, 0, s, mb); break;
    case 2: hipLaunchKernelGGL((k_voxel_combine_batch<2>), gl, bl, 0, s, mb); break;
    case 4: hipLaunchKernelGGL((k_voxel_combine_batch<4>), gl, bl, 0, s, mb); break;
    case 8: hipLaunchKernelGGL((k_voxel_combine_batch<8>), gl, bl, 0, s, mb); break;
    case 16: hipLaunchKernelGGL((k_voxel_combine_batch<16>), gl, bl, 0, s, mb); break;
    default: break;
    }
}

static void launch_leaf(int kind, const FrameParams &fp, const MapDev &md, int blocks, hipStream_t s)
{
    const dim3 gl(blocks), bl(kLeafThreads);
    if (kind <= 4) {
        // accumulating kernel with one set of accumulators per frame of the pass
        const int fr = fp.nsub <= 1 ? 1 : (fp.nsub == 2 ? 2 : (fp.nsub <= 4 ? 4 : 8));
        const int kmax = kind * 8;
#define SLIM_ACC(K, F) \
    if (kmax == K && fr == F) hipLaunchKernelGGL((k_leaf_acc<K, F>), gl, bl, 0, s, fp, md);
        SLIM_ACC(0, 1) SLIM_ACC(0, 2) SLIM_ACC(0, 4) SLIM_ACC(8, 1) SLIM_ACC(8, 2) SLIM_ACC(8, 4)
        SLIM_ACC(16, 1) SLIM_ACC(16, 2) SLIM_ACC(16, 4) SLIM_ACC(24, 1) SLIM_ACC(24, 2) SLIM_ACC(24, 4)
        SLIM_ACC(32, 1) SLIM_ACC(32, 2) SLIM_ACC(32, 4) SLIM_ACC(0, 8) SLIM_ACC(8, 8) SLIM_ACC(16, 8)
        SLIM_ACC(24, 8) SLIM_ACC(32, 8)
#undef SLIM_ACC
        return;
    }
    switch (kind) {
    case 5: hipLaunchKernelGGL((k_leaf_fuse<8, false, true>), gl, bl, 0, s, fp, md); break;
    case 6: hipLaunchKernelGGL((k_leaf_fuse<16, false, true>), gl, bl, 0, s, fp, md); break;
    case 7: hipLaunchKernelGGL((k_leaf_fuse<32, false, true>), gl, bl, 0, s, fp, md); break;
    case 16: hipLaunchKernelGGL((k_leaf_fuse<24, false, true>), gl, bl, 0, s, fp, md); break;
    case 9: hipLaunchKernelGGL((k_leaf_fuse<-1, false, false>), gl, bl, 0, s, fp, md); break;
    case 10: hipLaunchKernelGGL((k_leaf_fuse<-1, true, false>), gl, bl, 0, s, fp, md); break;
    case 11: hipLaunchKernelGGL((k_leaf_fuse<1, true, false>), gl, bl, 0, s, fp, md); break;
    case 12: hipLaunchKernelGGL((k_leaf_fuse<2, true, false>), gl, bl, 0, s, fp, md); break;
    case 13: hipLaunchKernelGGL((k_leaf_fuse<4, true, false>), gl, bl, 0, s, fp, md); break;
    case 14: hipLaunchKernelGGL((k_leaf_fuse<8, true, false>), gl, bl, 0, s, fp, md); break;
    case 15: hipLaunchKernelGGL((k_leaf_fuse<16, true, false>), gl, bl, 0, s, fp, md); break;
    default: hipLaunchKernelGGL((k_leaf_fuse<0, true, false>), gl, bl, 0, s, fp, md); break;
    }
}

static void launch_leaf_batch(int kind, const MapBatch &mb, int blocks, hipStream_t s)
{
    const dim3 gl(blocks), bl(kLeafThreads);
    switch (kind) {
    case 0: hipLaunchKernelGGL((k_leaf_acc_batch<0>), gl, bl, 0, s, mb); break;
    case 1: hipLaunchKernelGGL((k_leaf_acc_batch<8>), gl, bl, 0, s, mb); break;
    case 2: hipLaunchKernelGGL((k_leaf_acc_batch<16>), gl, bl, 0, s, mb); break;
    case 3: hipLaunchKernelGGL((k_leaf_acc_batch<24>), gl, bl, 0, s, mb); break;
    case 4: hipLaunchKernelGGL((k_leaf_acc_batch<32>), gl, bl, 0, s, mb); break;
    case 5: hipLaunchKernelGGL((k_leaf_fuse_batch<8, false, true>), gl, bl, 0, s, mb); break;
    case 6: hipLaunchKernelGGL((k_leaf_fuse_batch<16, false, true>), gl, bl, 0, s, mb); break;
    case 7: hipLaunchKernelGGL((k_leaf_fuse_batch<32, false, true>), gl, bl, 0, s, mb); break;
    case 16: hipLaunchKernelGGL((k_leaf_fuse_batch<24, false, true>), gl, bl, 0, s, mb); break;
    case 9: hipLaunchKernelGGL((k_leaf_fuse_batch<-1, false, false>), gl, bl, 0, s, mb); break;
    case 10: hipLaunchKernelGGL((k_leaf_fuse_batch<-1, true, false>), gl, bl, 0, s, mb); break;
    case 11: hipLaunchKernelGGL((k_leaf_fuse_batch<1, true, false>), gl, bl, 0, s, mb); break;
    case 12: hipLaunchKernelGGL((k_leaf_fuse_batch<2, true, false>), gl, bl, 0, s, mb); break;
    case 13: hipLaunchKernelGGL((k_leaf_fuse_batch<4, true, false>), gl, bl, 0, s, mb); break;
    case 14: hipLaunchKernelGGL((k_leaf_fuse_batch<8, true, false>), gl, bl, 0, s, mb); break;
    case 15: hipLaunchKernelGGL((k_leaf_fuse_batch<16, true, false>), gl, bl, 0, s, mb); break;
    default: hipLaunchKernelGGL((k_leaf_fuse_batch<0, true, false>), gl, bl, 0, s, mb); break;
    }
}

hipError_t launch_integrate(const FrameParams &fp, const MapDev &md_in, const LaunchShape &shape, hipStream_t s,
                            hipEvent_t *ev, const PassWalk *pw)
{
    MapDev md = md_in;
    md.leaf_blocks = shape.leaf_blocks;
    md.wave_pairs = shape.wave_pairs;
    md.slab_pairs = shape.slab_pairs;
    const int bw = (fp.n + kWalkThreads - 1) / kWalkThreads;
    auto rec = [&](int e) {
        if (ev) (void)hipEventRecord(ev[e], s);
    };
    rec(0);
    if (pw) {
        const int nb = pw->blk_start[pw->nframes];
        hipLaunchKernelGGL(k_ray_walk_emit_pass, dim3(nb > 0 ? nb : 1), dim3(kWalkThreads), 0, s, *pw, md);
    } else {
        hipLaunchKernelGGL(k_ray_walk_emit, dim3(bw > 0 ? bw : 1), dim3(kWalkThreads), 0, s, fp, md);
    }
    rec(1);
    rec(2);
    hipLaunchKernelGGL(k_leaf_plan, dim3(shape.plan_blocks), dim3(256), 0, s, fp, md);
    rec(3);
    rec(4);
    const long long want = ((long long)fp.n * fp.maxsteps + 255) / 256;
    const int bb = (int)std::max<long long>(1, std::min<long long>(want, shape.bucket_blocks));
    hipLaunchKernelGGL(k_pair_bucket, dim3(bb), dim3(256), 0, s, fp, md);
    rec(5);
    rec(6);
    const int kind = leaf_kernel_kind(fp);
    launch_leaf(kind, fp, md, shape.leaf_blocks, s);
    rec(7);
    rec(8);
    launch_voxel_combine(kind, fp, md, combine_blocks(kind, shape), s);
    rec(9);
    rec(10);
    hipLaunchKernelGGL(k_frame_commit, dim3(1), dim3(256), 0, s, fp, md);
    rec(11);
    return hipGetLastError();
}

hipError_t launch_walk(const FrameParams &fp, const MapDev &md, hipStream_t s, const PassWalk *pw)
{
    if (pw) {
        const int nb = pw->blk_start[pw->nframes];
        hipLaunchKernelGGL(k_ray_walk_emit_pass, dim3(nb > 0 ? nb : 1), dim3(kWalkThreads), 0, s, *pw, md);
        return hipGetLastError();
    }
    const int bw = (fp.n + kWalkThreads - 1) / kWalkThreads;
    hipLaunchKernelGGL(k_ray_walk_emit, dim3(bw > 0 ? bw : 1), dim3(kWalkThreads), 0, s, fp, md);
    return hipGetLastError();
}

hipError_t launch_after_walk(const FrameParams &fp, const MapDev &md_in, const LaunchShape &shape, hipStream_t s)
{
    MapDev md = md_in;
    md.leaf_blocks = shape.leaf_blocks;
    md.wave_pairs = shape.wave_pairs;
    md.slab_pairs = shape.slab_pairs;
    hipLaunchKernelGGL(k_leaf_plan, dim3(shape.plan_blocks), dim3(256), 0, s, fp, md);
    const long long want = ((long long)fp.n * fp.maxsteps + 255) / 256;
    const int bb = (int)std::max<long long>(1, std::min<long long>(want, shape.bucket_blocks));
    hipLaunchKernelGGL(k_pair_bucket, dim3(bb), dim3(256), 0, s, fp, md);
    const int kind = leaf_kernel_kind(fp);
    launch_leaf(kind, fp, md, shape.leaf_blocks, s);
    launch_voxel_combine(kind, fp, md, combine_blocks(kind, shape), s);
    hipLaunchKernelGGL(k_frame_commit, dim3(1), dim3(256), 0, s, fp, md);
    return hipGetLastError();
}

hipError_t launch_integrate_batched(const MapBatch &mb, const BatchPlan &plan, const LaunchShape &shape,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(k_ray_walk_emit_batch, dim3(std::max(plan.walk_blocks, 1)), dim3(kWalkThreads), 0, s, mb);
    hipLaunchKernelGGL(k_leaf_plan_batch, dim3(plan.plan_blocks), dim3(256), 0, s, mb);
    hipLaunchKernelGGL(k_pair_bucket_batch, dim3(plan.bucket_blocks), dim3(256), 0, s, mb);
    for (int g = 0; g < plan.ngroups; ++g) {
        MapBatch sub = mb;
        sub.subset = mb.subset + plan.group_begin[g];
        sub.nsubset = plan.group_size[g];
        sub.part_first = mb.part_first + plan.leaf_part[g];
        launch_leaf_batch(plan.group_kind[g], sub, plan.leaf_blocks[g], s);
        sub.part_first = mb.part_first + plan.comb_part[g];
        if (plan.comb_blocks[g] > 0) launch_voxel_combine_batch(plan.group_kind[g], sub, plan.comb_blocks[g], s);
    }
    hipLaunchKernelGGL(k_frame_commit_batch, dim3(plan.nmaps), dim3(256), 0, s, mb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// map loss and backward (differentiation workload)
// ---------------------------------------------------------------------------

// Record of the voxel with integer key (kx, ky, kz), or -1 if it has W = 0.
__device__ __forceinline__ long long voxel_record(const MapDev &md, int kx, int ky, int kz)
{
    const int slot = map_find(md, pack_leaf(kx >> 3, ky >> 3, kz >> 3));
    if (slot < 0) return -1;
    const int off = ((kx & 7) << 6) | ((ky & 7) << 3) | (kz & 7);
    if (!((md.leaf_occ[(size_t)slot * kMaskWords + (off >> 5)] >> (off & 31)) & 1u)) return -1;
    return (long long)md.leaf_page[(size_t)slot * kLeafPages + (off >> 6)] * kPageVoxels + (off & (kPageVoxels - 1));
}

// Record of the voxel holding world point (x, y, z): floor(x / vs), binary32.
__device__ __forceinline__ long long point_record(const MapDev &md, float vs, float x, float y, float z)
{
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) return -1;
    const float fx = floorf(x / vs), fy = floorf(y / vs), fz = floorf(z / vs);
    const float lim = (float)kKeyLimit;
    if (!(fabsf(fx) < lim && fabsf(fy) < lim && fabsf(fz) < lim)) return -1;
    return voxel_record(md, (int)fx, (int)fy, (int)fz);
}

// Block sum of one float per thread in a fixed tree order (blockDim.x = 256).
__device__ __forceinline__ float block_sum(float v, float *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int d = kLossThreads / 2; d > 0; d >>= 1) {
        if (threadIdx.x < (unsigned)d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

// Clears the sample counts and the adjoints of every record in use, so that a
// voxel the loss does not list (or lists with a label outside [0, K)) carries
// zero adjoints into the backward.
__global__ __launch_bounds__(256) void k_loss_clear(MapDev md, LossParams lp)
{
    const size_t n = (size_t)md.st->pages_used * kPageVoxels;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) lp.adj_cnt[i] = 0;
    // adj_stride is a multiple of 4 floats
    float4 *a4 = (float4 *)lp.adj;
    const size_t n4 = n * (size_t)(lp.adj_stride / 4);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += stride)
        a4[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Surface samples: per voxel count (integer, so order-free) and block partials
// of |D| and of the number of samples that land in the map.
__global__ __launch_bounds__(kLossThreads) void k_loss_samples(FrameParams fp, MapDev md, LossParams lp)
{
    __shared__ float red[kLossThreads];
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    float a = 0.0f, c = 0.0f;
    if (i < lp.s) {
        const long long rec = point_record(md, fp.vs, lp.samples[3 * i], lp.samples[3 * i + 1], lp.samples[3 * i + 2]);
        if (rec >= 0) {
            atomicAdd(&lp.adj_cnt[rec], 1);
            a = fabsf(md.vox[(size_t)rec * md.rec_stride]);
            c = 1.0f;
        }
    }
    a = block_sum(a, red);
    c = block_sum(c, red);
    if (threadIdx.x == 0) {
        lp.part[blockIdx.x] = a;
        lp.part_cnt[blockIdx.x] = (int)c;
    }
}

// Voxels: cross-entropy of the Dirichlet predictive (Eq. (7)) at the true class,
// adjoints dL/dc and dL/dD, block partials of the cross-entropy.
__global__ __launch_bounds__(kLossThreads) void k_loss_voxels(FrameParams fp, MapDev md, LossParams lp, int nsb)
{
    __shared__ float red[kLossThreads];
    __shared__ int s_mp;
    if (threadIdx.x == 0) {
        int mp = 0;
        for (int b = 0; b < nsb; ++b) mp += lp.part_cnt[b];
        s_mp = mp;
    }
    __syncthreads();
    const float inv_m = 1.0f / (float)lp.m, inv_mp = s_mp > 0 ? 1.0f / (float)s_mp : 0.0f;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int K = fp.K;
    float ce = 0.0f;
    if (i < lp.m) {
        const long long rec = voxel_record(md, lp.keys[3 * i], lp.keys[3 * i + 1], lp.keys[3 * i + 2]);
        const int y = lp.labels[i];
        if (rec >= 0) {
            const float *R = md.vox + (size_t)rec * md.rec_stride;
            float *A = lp.adj + (size_t)rec * lp.adj_stride;
            // a label outside [0, K) adds no cross-entropy term (dL/dc = 0);
            // the voxel's surface samples still count
            if (y >= 0 && y < K) {
                float tot = (float)K * lp.alpha0;
                for (int k = 0; k < K; ++k) tot += R[2 + k];
                const float ay = lp.alpha0 + R[2 + y];
                ce = -logf(ay / tot);
                const float g = inv_m / tot;
                for (int k = 0; k < K; ++k) A[k] = k == y ? g - inv_m / ay : g;
            }
            const float D = R[0];
            const float sg = D > 0.0f ? 1.0f : (D < 0.0f ? -1.0f : 0.0f);
            A[K] = sg * (float)lp.adj_cnt[rec] * inv_mp;
        }
    }
    ce = block_sum(ce, red);
    if (threadIdx.x == 0) lp.part[nsb + blockIdx.x] = ce;
}

__global__ __launch_bounds__(256) void k_loss_final(LossParams lp, int nsb, int nvb)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float l1 = 0.0f, ce = 0.0f;
    int mp = 0;
    for (int b = 0; b < nsb; ++b) {
        l1 += lp.part[b];
        mp += lp.part_cnt[b];
    }
    for (int b = 0; b < nvb; ++b) ce += lp.part[nsb + b];
    const float t_ce = ce / (float)lp.m, t_l1 = mp > 0 ? l1 / (float)mp : 0.0f;
    lp.loss[0] = t_ce + t_l1;
    lp.loss[1] = t_ce;
    lp.loss[2] = t_l1;
}

hipError_t launch_loss(const FrameParams &fp, const MapDev &md, const LossParams &lp, hipStream_t s)
{
    const int nsb = (int)((lp.s + kLossThreads - 1) / kLossThreads);
    const int nvb = (int)((lp.m + kLossThreads - 1) / kLossThreads);
    hipLaunchKernelGGL(k_loss_clear, dim3(1024), dim3(256), 0, s, md, lp);
    if (nsb > 0) hipLaunchKernelGGL(k_loss_samples, dim3(nsb), dim3(kLossThreads), 0, s, fp, md, lp);
    if (nvb > 0) hipLaunchKernelGGL(k_loss_voxels, dim3(nvb), dim3(kLossThreads), 0, s, fp, md, lp, nsb);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, lp, nsb, nvb);
    return hipGetLastError();
}

// One lane per ray: recompute the band walk, gather the adjoints of the voxels
// it observed, and chain them through the softmax and the clamp.
template <int KMAX>
__global__ __launch_bounds__(256) void k_backward_rays(FrameParams fp, MapDev md, LossParams lp,
                                                       const float *grad_scale, float *grad_logits,
                                                       float *grad_ranges)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= fp.n) return;
    const int K = fp.K;
    float G[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) G[k] = 0.0f;
    float gr = 0.0f;
    Ray ry;
    float x, y, z;
    load_point(fp, i, x, y, z);
    bool valid = make_ray(fp, x, y, z, ry);
    if (valid) {
        bool inrange = true;
        unsigned long long cur = kEmptyKey;
        int slot = -1;
        const bool started = band_walk(fp, ry, [&](int cx, int cy, int cz) {
            const int kx = fp.a[0] + cx, ky = fp.a[1] + cy, kz = fp.a[2] + cz;
            if (!(key_ok(kx) && key_ok(ky) && key_ok(kz))) {
                inrange = false;
                return;
            }
            const float sdf = cell_sdf(fp, ry, cx, cy, cz);
            if (!(sdf > -fp.tau) || !inrange) return;
            const unsigned long long lk = pack_leaf(kx >> 3, ky >> 3, kz >> 3);
            if (lk != cur) {
                cur = lk;
                slot = map_find(md, lk);
            }
            if (slot < 0) return;
            const int off = ((kx & 7) << 6) | ((ky & 7) << 3) | (kz & 7);
            const int page = md.leaf_page[(size_t)slot * kLeafPages + (off >> 6)];
            if (page < 0) return;  // not a voxel of this map (inputs differ from the integrated ones)
            const long long rec = (long long)page * kPageVoxels + (off & (kPageVoxels - 1));
            const float *A = lp.adj + (size_t)rec * lp.adj_stride;
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < K) G[k] += A[k];
            // a voxel no loss sample landed in has a zero adjoint (and may be an
            // unobserved record of an observed slab, W = 0)
            if (sdf < fp.tau && A[K] != 0.0f) gr += A[K] / md.vox[(size_t)rec * md.rec_stride + 1];
        });
        valid = started && inrange;
    }
    const float sc = grad_scale ? grad_scale[0] : 1.0f;
    float l[KMAX];
    float mx = -INFINITY;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        l[k] = k < K ? ((const float *)fp.sem)[(size_t)i * K + k] : -INFINITY;
        mx = fmaxf(mx, l[k]);
    }
    float den = 0.0f;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        l[k] = k < K ? expf(l[k] - mx) : 0.0f;
        den += l[k];
    }
    float pg = 0.0f;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        l[k] /= den;
        pg += l[k] * G[k];
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (k < K) grad_logits[(size_t)i * K + k] = valid ? sc * l[k] * (G[k] - pg) : 0.0f;
    grad_ranges[i] = valid ? sc * gr : 0.0f;
}

hipError_t launch_backward(const FrameParams &fp, const MapDev &md, const LossParams &lp, const float *grad_scale,
                           float *grad_logits, float *grad_ranges, hipStream_t s)
{
    const int b = (fp.n + 255) / 256;
    if (b == 0) return hipGetLastError();
    if (fp.K > 16) hipLaunchKernelGGL(k_backward_rays<32>, dim3(b), dim3(256), 0, s, fp, md, lp, grad_scale, grad_logits, grad_ranges);
    else if (fp.K > 8) hipLaunchKernelGGL(k_backward_rays<16>, dim3(b), dim3(256), 0, s, fp, md, lp, grad_scale, grad_logits, grad_ranges);
    else hipLaunchKernelGGL(k_backward_rays<8>, dim3(b), dim3(256), 0, s, fp, md, lp, grad_scale, grad_logits, grad_ranges);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reset, extract, query
// ---------------------------------------------------------------------------

__global__ void k_fill_u64(unsigned long long *p, size_t n, unsigned long long v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_reset_state(DevState *st, FrameState *fs)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (st) {
            DevState z = {};
            *st = z;
        }
        FrameState f = {};
        *fs = f;
    }
}

hipError_t launch_reset(const MapDev &md, hipStream_t s)
{
    const size_t cap = (size_t)md.hmask + 1;
    // free slots: key kEmptyKey (slot and padding all ones, never read)
    hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, (unsigned long long *)md.htab, 2 * cap, kEmptyKey);
    hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, md.skeys, cap, kEmptyKey);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, md.pos_count, cap, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, md.pos_slab, cap, 0u);
    hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, md.st, md.fs);
    return hipGetLastError();
}

// Clears a second staging buffer (its table, counts and frame counters).
hipError_t launch_reset_staging(const MapDev &md, hipStream_t s)
{
    const size_t cap = (size_t)md.hmask + 1;
    hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, md.skeys, cap, kEmptyKey);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, md.pos_count, cap, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, md.pos_slab, cap, 0u);
    hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, (DevState *)nullptr, md.fs);
    return hipGetLastError();
}

__device__ __forceinline__ uint32_t bits_below(const uint32_t *mask, uint32_t o)
{
    uint32_t r = 0;
    for (uint32_t w = 0; w < (o >> 5); ++w) r += __popc(mask[w]);
    return r + __popc(mask[o >> 5] & ((1u << (o & 31)) - 1u));
}

__global__ void k_collect_leaves(const MapDev md, long long nleaves, unsigned long long *keys, int32_t *slots)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nleaves;
         i += (long long)gridDim.x * blockDim.x) {
        keys[i] = md.leaf_key[i];
        slots[i] = (int32_t)i;
    }
}

// One compare-exchange step of a bitonic network over n elements (virtual
// +infinity beyond n) in global memory.  The first step of each stage compares
// mirrored positions, so every block sorts ascending.
__global__ void k_bitonic_step(unsigned long long *keys, int32_t *vals, long long n, long long k, long long d,
                               int mirrored, long long half)
{
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < half;
         t += (long long)gridDim.x * blockDim.x) {
        long long a, b;
        if (mirrored) {
            const long long hk = k >> 1, blk = t / hk, w = t % hk;
            a = blk * k + w;
            b = blk * k + k - 1 - w;
        } else {
            a = (t / d) * 2 * d + (t % d);
            b = a + d;
        }
        if (b < n && keys[b] < keys[a]) {
            const unsigned long long kt = keys[a];
            keys[a] = keys[b];
            keys[b] = kt;
            const int32_t vt = vals[a];
            vals[a] = vals[b];
            vals[b] = vt;
        }
    }
}

// Exclusive prefix sum of the voxel counts of the sorted leaves (single
// workgroup; extraction is not on the integration path).
__global__ __launch_bounds__(1024) void k_leaf_offsets(const MapDev md, long long nleaves, const int32_t *slots,
                                                       uint32_t *offsets)
{
    __shared__ uint32_t s_part[1024];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (long long b = 0; b < nleaves; b += 1024) {
        const long long i = b + threadIdx.x;
        uint32_t c = 0;
        if (i < nleaves)
            for (int w = 0; w < kMaskWords; ++w) c += __popc(md.leaf_occ[(size_t)slots[i] * kMaskWords + w]);
        s_part[threadIdx.x] = c;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const uint32_t v = threadIdx.x >= (unsigned)d ? s_part[threadIdx.x - d] : 0u;
            __syncthreads();
            s_part[threadIdx.x] += v;
            __syncthreads();
        }
        if (i < nleaves) offsets[i] = s_carry + s_part[threadIdx.x] - c;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry += s_part[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_extract(const MapDev md, long long nleaves, int nsem, const int32_t *slots,
                                                 const uint32_t *offsets, int32_t *keys, float *d, float *w,
                                                 float *sem)
{
    for (long long j = blockIdx.x; j < nleaves; j += gridDim.x) {
        const int slot = slots[j];
        const unsigned long long lk = md.leaf_key[slot];
        const int lx = (int)((lk >> 36) & 0x3FFFF) - kLeafBias;
        const int ly = (int)((lk >> 18) & 0x3FFFF) - kLeafBias;
        const int lz = (int)(lk & 0x3FFFF) - kLeafBias;
        const uint32_t *occ = md.leaf_occ + (size_t)slot * kMaskWords;
        for (int t = threadIdx.x; t < kLeafVoxels; t += blockDim.x) {
            if (!((occ[t >> 5] >> (t & 31)) & 1u)) continue;
            const size_t o = (size_t)offsets[j] + bits_below(occ, (uint32_t)t);
            const long long rec =
                (long long)md.leaf_page[(size_t)slot * kLeafPages + (t >> 6)] * kPageVoxels + (t & (kPageVoxels - 1));
            const float *R = md.vox + (size_t)rec * md.rec_stride;
            keys[3 * o + 0] = lx * 8 + (t >> 6);
            keys[3 * o + 1] = ly * 8 + ((t >> 3) & 7);
            keys[3 * o + 2] = lz * 8 + (t & 7);
            d[o] = R[0];
            w[o] = R[1];
            if (sem)
                for (int k = 0; k < nsem; ++k) sem[o * nsem + k] = R[2 + k];
        }
    }
}

hipError_t launch_extract(const MapDev &md, int nsem, long long nleaves, unsigned long long *tmp_keys,
                          int32_t *tmp_slots, uint32_t *tmp_offsets, int32_t *keys, float *d, float *w, float *sem,
                          hipStream_t s)
{
    if (nleaves <= 0) return hipGetLastError();
    hipLaunchKernelGGL(k_collect_leaves, dim3(256), dim3(256), 0, s, md, nleaves, tmp_keys, tmp_slots);
    long long np2 = 1;
    while (np2 < nleaves) np2 <<= 1;
    const long long half = np2 >> 1;
    const int blocks = (int)std::min<long long>((half + 255) / 256 + 1, 4096);
    for (long long k = 2; k <= np2; k <<= 1) {
        hipLaunchKernelGGL(k_bitonic_step, dim3(blocks), dim3(256), 0, s, tmp_keys, tmp_slots, nleaves, k, 0LL, 1,
                           half);
        for (long long dd = k >> 2; dd > 0; dd >>= 1)
            hipLaunchKernelGGL(k_bitonic_step, dim3(blocks), dim3(256), 0, s, tmp_keys, tmp_slots, nleaves, k, dd, 0,
                               half);
    }
    hipLaunchKernelGGL(k_leaf_offsets, dim3(1), dim3(1024), 0, s, md, nleaves, tmp_slots, tmp_offsets);
    hipLaunchKernelGGL(k_extract, dim3((unsigned)std::min<long long>(nleaves, 8192)), dim3(256), 0, s, md, nleaves,
                       nsem, tmp_slots, tmp_offsets, keys, d, w, sem);
    return hipGetLastError();
}

// Scratch of the allocation-free extract (slim_extract_noalloc): the leaves'
// keys, then their slots, then their voxel offsets, for at most
// kNoAllocMaxLeaves leaves.  Each GPU the library runs on holds its own copy
// until the process ends.  In host code `scratch` names a host-side stand-in:
// kernels get the device address that noalloc_scratch_setup resolved.
static __device__ __align__(256) unsigned char scratch[kNoAllocMaxLeaves * 16];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocMaxDevices];
}  // namespace

hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Record of the voxel holding world point (x, y, z), floor(x / vs) in binary32;
// -1 if unobserved, non-finite or out of the key range.
__device__ __forceinline__ long long lookup_point(const MapDev &md, float vs, float x, float y, float z)
{
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) return -1;
    const float fx = floorf(x / vs), fy = floorf(y / vs), fz = floorf(z / vs);
    const float lim = (float)kKeyLimit;
    if (!(fabsf(fx) < lim && fabsf(fy) < lim && fabsf(fz) < lim)) return -1;
    const int kx = (int)fx, ky = (int)fy, kz = (int)fz;
    const int slot = map_find(md, pack_leaf(kx >> 3, ky >> 3, kz >> 3));
    if (slot < 0) return -1;
    const int off = ((kx & 7) << 6) | ((ky & 7) << 3) | (kz & 7);
    if (!((md.leaf_occ[(size_t)slot * kMaskWords + (off >> 5)] >> (off & 31)) & 1u)) return -1;
    return (long long)md.leaf_page[(size_t)slot * kLeafPages + (off >> 6)] * kPageVoxels + (off & (kPageVoxels - 1));
}

__global__ __launch_bounds__(256) void k_query(const MapDev md, int nsem, float vs, const float *xyz, long long m,
                                               float *d, float *w, float *sem)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x) {
        const long long rec = lookup_point(md, vs, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
        if (rec >= 0) {
            const float *R = md.vox + (size_t)rec * md.rec_stride;
            d[i] = R[0];
            w[i] = R[1];
            if (sem)
                for (int k = 0; k < nsem; ++k) sem[i * nsem + k] = R[2 + k];
        } else {
            d[i] = 0.0f;
            w[i] = 0.0f;
            if (sem)
                for (int k = 0; k < nsem; ++k) sem[i * nsem + k] = 0.0f;
        }
    }
}

hipError_t launch_query(const MapDev &md, int nsem, float vs, const float *xyz, long long m, float *d, float *w,
                        float *sem, hipStream_t s)
{
    if (m <= 0) return hipGetLastError();
    const int blocks = (int)std::min<long long>((m + 255) / 256, 4096);
    hipLaunchKernelGGL(k_query, dim3(blocks), dim3(256), 0, s, md, nsem, vs, xyz, m, d, w, sem);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// semantic read-out: Eq. (7), Eq. (15), prototype softmax and threshold
// ---------------------------------------------------------------------------

constexpr int kPredictMaxC = 1024;  // classes or prototypes

// First index of the largest value across the wave: (v, i) pairs, larger v
// wins, equal v the smaller i.
__device__ __forceinline__ void wave_argmax(float &v, int &i)
{
    for (int d = 32; d > 0; d >>= 1) {
        const float ov = __shfl_xor(v, d, 64);
        const int oi = __shfl_xor(i, d, 64);
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    }
}

// One wave per query point.  sims: per-wave LDS row of similarities (open set).
__global__ __launch_bounds__(256) void k_predict(const MapDev md, const PredictParams pp, const float *xyz,
                                                 long long m, float *prob, int32_t *label, float *var)
{
    __shared__ float sims[4][kPredictMaxC];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const long long nwaves = (long long)gridDim.x * (blockDim.x >> 6);
    const bool open = pp.mode == SLIM_SEM_OPEN || pp.mode == SLIM_SEM_OPEN_LAST;
    for (long long q = blockIdx.x * (long long)(blockDim.x >> 6) + wv; q < m; q += nwaves) {
        const long long rec = lookup_point(md, pp.vs, xyz[3 * q], xyz[3 * q + 1], xyz[3 * q + 2]);
        const float *R = rec >= 0 ? md.vox + (size_t)rec * md.rec_stride : nullptr;
        float best = -INFINITY;
        int arg = 0x7FFFFFFF;
        if (pp.mode == SLIM_SEM_CLOSED) {
            // Eq. (7): the Dirichlet predictive
            float part = 0.0f;
            for (int k = lane; k < pp.K; k += 64) part += R ? R[2 + k] : 0.0f;
            const float den = (float)pp.K * pp.alpha0 + wave_sum(part);
            for (int k = lane; k < pp.K; k += 64) {
                const float p = (pp.alpha0 + (R ? R[2 + k] : 0.0f)) / den;
                if (prob) prob[q * pp.K + k] = p;
                if (p > best) {
                    best = p;
                    arg = k;
                }
            }
        } else if (pp.mode == SLIM_SEM_CLOSED_LAST) {
            const int cls = R ? (int)R[2] : -1;
            for (int k = lane; k < pp.K; k += 64) {
                const float p = k == cls ? 1.0f : 0.0f;
                if (prob) prob[q * pp.K + k] = p;
                if (p > best) {
                    best = p;
                    arg = k;
                }
            }
        } else if (open && R) {
            // cosine similarity of the predictive mean with every prototype
            float n2 = 0.0f;
            for (int d = lane; d < pp.L; d += 64) n2 += R[2 + d] * R[2 + d];
            const float nm = sqrtf(wave_sum(n2));
            for (int j = 0; j < pp.P; ++j) {
                const float *Q = pp.protos + (size_t)j * pp.L;
                float dot = 0.0f, q2 = 0.0f;
                for (int d = lane; d < pp.L; d += 64) {
                    const float qd = Q[d];
                    dot += R[2 + d] * qd;
                    q2 += qd * qd;
                }
                dot = wave_sum(dot);
                q2 = wave_sum(q2);
                if (lane == 0) sims[wv][j] = dot / (nm * sqrtf(q2)) * pp.inv_temp;
            }
            wave_sync();
            float mx = -INFINITY;
            for (int j = lane; j < pp.P; j += 64) mx = fmaxf(mx, sims[wv][j]);
            mx = wave_max(mx);
            float es = 0.0f;
            for (int j = lane; j < pp.P; j += 64) es += expf(sims[wv][j] - mx);
            const float den = wave_sum(es);
            for (int j = lane; j < pp.P; j += 64) {
                const float p = expf(sims[wv][j] - mx) / den;
                if (prob) prob[q * pp.P + j] = p;
                if (p > best) {
                    best = p;
                    arg = j;
                }
            }
            wave_sync();
        } else if (open) {
            for (int j = lane; j < pp.P; j += 64)
                if (prob) prob[q * pp.P + j] = 0.0f;
        }
        if (var && pp.mode == SLIM_SEM_OPEN) {
            // Eq. (15) with lambda = 2 nu = W: variance 2 beta (W + 1) / (W (W - 2)) for W > 2
            const float W = R ? R[1] : 0.0f;
            for (int d = lane; d < pp.L; d += 64)
                var[q * pp.L + d] = W > 2.0f ? 2.0f * R[2 + pp.L + d] * (W + 1.0f) / (W * (W - 2.0f)) : NAN;
        }
        wave_argmax(best, arg);
        if (label && lane == 0) label[q] = (R && best >= pp.threshold) ? arg : -1;
    }
}

hipError_t launch_predict(const MapDev &md, const PredictParams &pp, const float *xyz, long long m, float *prob,
                          int32_t *label, float *var, hipStream_t s)
{
    if (m <= 0) return hipGetLastError();
    const int blocks = (int)std::min<long long>((m + 3) / 4, 65536);
    hipLaunchKernelGGL(k_predict, dim3(blocks), dim3(256), 0, s, md, pp, xyz, m, prob, label, var);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// render: first surface per pixel (the map-viewing role of Sec. III-E)
// ---------------------------------------------------------------------------

// One thread per pixel.  The ray is formed as a sensor point at unit depth is
// (same binary32 operations), walked with the integration walk's stepping rule
// over [t0, t1], and stops at the first pair of consecutive observed cells with
// D > 0 then D <= 0; the depth interpolates the cell centres' projections onto
// the ray linearly in D.  The leaf slot is cached while the walk stays in a leaf.
__global__ __launch_bounds__(256) void k_render(const MapDev md, const RenderParams rp, float *depth, int32_t *key,
                                                int32_t *label)
{
    const int px = blockIdx.x * 64 + (threadIdx.x & 63), py = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (px >= rp.width || py >= rp.height) return;
    const long long i = (long long)py * rp.width + px;
    float out_d = NAN;
    int ok[3] = {0, 0, 0}, out_l = -1;
    const float dc0 = ((float)px - rp.cx) / rp.fx, dc1 = ((float)py - rp.cy) / rp.fy, dc2 = 1.0f;
    float p[3], u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        p[a] = fmaf(rp.R[3 * a + 0], dc0, fmaf(rp.R[3 * a + 1], dc1, fmaf(rp.R[3 * a + 2], dc2, rp.t[a])));
    const float d0 = p[0] - rp.t[0], d1 = p[1] - rp.t[1], d2 = p[2] - rp.t[2];
    const float r = sqrtf(fmaf(d2, d2, fmaf(d1, d1, d0 * d0)));
    if (r > 0.0f && isfinite(r)) {
        u[0] = d0 / r;
        u[1] = d1 / r;
        u[2] = d2 / r;
        const float vs = rp.vs, t0 = rp.t0, h = 0.5f * vs;
        int c[3], stp[3];
        float tm[3], td[3];
        bool start_ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float s = fmaf(t0, u[a], rp.t[a]);
            const float fc = floorf(s / vs);
            start_ok = start_ok && fabsf(fc) < kCellLimit;
            c[a] = fabsf(fc) < kCellLimit ? (int)fc : 0;
            if (u[a] > 0.0f) {
                stp[a] = 1;
                tm[a] = t0 + fmaf((float)(c[a] + 1), vs, -s) / u[a];
                td[a] = vs / u[a];
            } else if (u[a] < 0.0f) {
                stp[a] = -1;
                tm[a] = t0 + fmaf((float)c[a], vs, -s) / u[a];
                td[a] = -vs / u[a];
            } else {
                stp[a] = 0;
                tm[a] = INFINITY;
                td[a] = INFINITY;
            }
        }
        unsigned long long cur = kEmptyKey;
        int slot = -1;
        bool have_prev = false;
        float Dp = 0.0f, sp = 0.0f;
        for (int it = 0; it < (start_ok ? rp.maxsteps : 0); ++it) {
            const int kx = rp.a[0] + c[0], ky = rp.a[1] + c[1], kz = rp.a[2] + c[2];
            if (!(key_ok(kx) && key_ok(ky) && key_ok(kz))) break;
            const unsigned long long lk = pack_leaf(kx >> 3, ky >> 3, kz >> 3);
            if (lk != cur) {
                cur = lk;
                slot = map_find(md, lk);
            }
            long long rec = -1;
            if (slot >= 0) {
                const int off = ((kx & 7) << 6) | ((ky & 7) << 3) | (kz & 7);
                if ((md.leaf_occ[(size_t)slot * kMaskWords + (off >> 5)] >> (off & 31)) & 1u)
                    rec = (long long)md.leaf_page[(size_t)slot * kLeafPages + (off >> 6)] * kPageVoxels +
                          (off & (kPageVoxels - 1));
            }
            if (rec < 0) {
                have_prev = false;
            } else {
                const float *R = md.vox + (size_t)rec * md.rec_stride;
                const float D = R[0];
                const float qx = fmaf((float)c[0], vs, h) - rp.t[0];
                const float qy = fmaf((float)c[1], vs, h) - rp.t[1];
                const float qz = fmaf((float)c[2], vs, h) - rp.t[2];
                const float sk = fmaf(qz, u[2], fmaf(qy, u[1], qx * u[0]));
                if (have_prev && Dp > 0.0f && D <= 0.0f) {
                    out_d = sp + (sk - sp) * (Dp / (Dp - D));
                    ok[0] = kx;
                    ok[1] = ky;
                    ok[2] = kz;
                    if (rp.mode == SLIM_SEM_CLOSED) {
                        float best = R[2];
                        out_l = 0;
                        for (int k = 1; k < rp.K; ++k)
                            if (R[2 + k] > best) {
                                best = R[2 + k];
                                out_l = k;
                            }
                    } else if (rp.mode == SLIM_SEM_CLOSED_LAST) {
                        out_l = (int)R[2];
                    }
                    break;
                }
                have_prev = true;
                Dp = D;
                sp = sk;
            }
            const bool xy = tm[0] <= tm[1];
            const int ax = xy ? (tm[0] <= tm[2] ? 0 : 2) : (tm[1] <= tm[2] ? 1 : 2);
            const float tnext = ax == 0 ? tm[0] : (ax == 1 ? tm[1] : tm[2]);
            if (tnext > rp.t1) break;
            if (ax == 0) { c[0] += stp[0]; tm[0] += td[0]; }
            else if (ax == 1) { c[1] += stp[1]; tm[1] += td[1]; }
            else { c[2] += stp[2]; tm[2] += td[2]; }
        }
    }
    depth[i] = out_d;
    if (key) {
        key[3 * i + 0] = ok[0];
        key[3 * i + 1] = ok[1];
        key[3 * i + 2] = ok[2];
    }
    if (label) label[i] = out_l;
}

hipError_t launch_render(const MapDev &md, const RenderParams &rp, float *depth, int32_t *key, int32_t *label,
                         hipStream_t s)
{
    if (rp.width <= 0 || rp.height <= 0) return hipGetLastError();
    const dim3 grid((rp.width + 63) / 64, (rp.height + 3) / 4);
    hipLaunchKernelGGL(k_render, grid, dim3(256), 0, s, md, rp, depth, key, label);
    return hipGetLastError();
}

}  // namespace slim
