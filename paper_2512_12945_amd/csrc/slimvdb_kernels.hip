// HIP kernels of the semantic TSDF integrator (gfx950, wave64).
//
// One frame runs as four kernels on the map's stream:
//   1. ray_walk_emit  one lane per point: pose application, ray, band, voxel
//                     walk (Sec. III-A), truncation gate; leaf runs of each
//                     ray are staged (frame-local leaf table) and every kept
//                     (voxel, point) observation is written as a pair.
//   2. leaf_plan      one lane per touched leaf: find it in the map, count
//                     its new voxels, allocate its pair bucket.
//   3. pair_bucket    one lane per pair: scatter into its leaf's bucket.
//   4. leaf_apply     one workgroup per touched leaf: sort the bucket by
//                     (voxel offset, point index) in LDS, reduce each voxel's
//                     observations in point order, and combine them with the
//                     stored state: Eq. (1)-(2) for D and W, Eq. (6) for the
//                     class counts, Eqs. (11)-(14) with lambda = 2 nu = W for
//                     the open-set mean and beta.  Its last workgroup commits
//                     the frame's counters.
// Capacity is checked in leaf_apply before any map write, so a frame that does
// not fit changes nothing.  No floating-point atomics are used: each voxel's
// sums are formed by one lane in point order, so results are bitwise
// repeatable and independent of launch shapes.
//
// The geometric decision path (pose, ray, walk, gate) is a fixed sequence of
// binary32 operations; build with -ffp-contract=off so that only the fmaf()
// calls written here fuse, and with correctly rounded division and sqrt.

#include <hip/hip_runtime.h>

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

__device__ __forceinline__ unsigned long long load_key(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Slot of a leaf in the map's table, or -1.
__device__ int32_t map_find(const MapDev &md, unsigned long long key)
{
    uint32_t h = leaf_hash(key, md.hmask);
    for (uint32_t probe = 0; probe <= md.hmask; ++probe) {
        unsigned long long k = md.hkeys[h];
        if (k == key) return md.hvals[h];
        if (k == kEmptyKey) return -1;
        h = (h + 1) & md.hmask;
    }
    return -1;
}

// Inserts a leaf known to be absent.  The table is at most half full.
__device__ void map_insert(const MapDev &md, unsigned long long key, int32_t slot)
{
    uint32_t h = leaf_hash(key, md.hmask);
    for (uint32_t probe = 0; probe <= md.hmask; ++probe) {
        unsigned long long prev = atomicCAS(&md.hkeys[h], kEmptyKey, key);
        if (prev == kEmptyKey) {
            md.hvals[h] = slot;
            return;
        }
        h = (h + 1) & md.hmask;
    }
}

// Staging-table position of a leaf touched by this frame, inserting it on
// first sight.  kNoPos if the table is full.
__device__ uint32_t stage_leaf(const MapDev &md, unsigned long long key)
{
    uint32_t h = leaf_hash(key, md.hmask);
    for (uint32_t probe = 0; probe <= md.hmask; ++probe) {
        unsigned long long cur = load_key(&md.skeys[h]);
        if (cur == key) return h;
        if (cur == kEmptyKey) {
            unsigned long long prev = atomicCAS(&md.skeys[h], kEmptyKey, key);
            if (prev == kEmptyKey) {
                uint32_t j = atomicAdd(&md.st->n_touched, 1u);
                md.touched[j] = h;
                return h;
            }
            if (prev == key) return h;
        }
        h = (h + 1) & md.hmask;
    }
    return kNoPos;
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

// Wave-aggregated atomicAdd: every lane of the wave must call it.  Returns
// the lane's exclusive offset into the reserved range.
__device__ __forceinline__ uint32_t wave_reserve(unsigned int *counter, uint32_t v)
{
    uint32_t incl = wave_incl_scan(v);
    uint32_t total = __shfl(incl, 63, 64);
    uint32_t base = 0;
    if (lane_id() == 63 && total) base = atomicAdd(counter, total);
    base = __shfl(base, 63, 64);
    return base + incl - v;
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

// Amanatides-Woo walk over the band of the ray from the sensor origin
// (fp.t).  Calls visit(cx, cy, cz) per cell (anchor-relative).  Ties between
// axes step the lowest axis first, one axis per step; the walk stops when the
// next boundary lies beyond t1, or after maxsteps cells.
template <class Visit>
__device__ __forceinline__ void band_walk(const FrameParams &fp, const Ray &ry, Visit &&visit)
{
    const float vs = fp.vs, t0 = ry.t0;
    int c[3], stp[3];
    float tm[3], td[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float s = fmaf(t0, ry.u[a], fp.t[a]);
        c[a] = (int)floorf(s / vs);
        if (ry.u[a] > 0.0f) {
            stp[a] = 1;
            tm[a] = t0 + fmaf((float)(c[a] + 1), vs, -s) / ry.u[a];
            td[a] = vs / ry.u[a];
        } else if (ry.u[a] < 0.0f) {
            stp[a] = -1;
            tm[a] = t0 + fmaf((float)c[a], vs, -s) / ry.u[a];
            td[a] = -vs / ry.u[a];
        } else {
            stp[a] = 0;
            tm[a] = INFINITY;
            td[a] = INFINITY;
        }
    }
    for (int it = 0; it < fp.maxsteps; ++it) {
        visit(c[0], c[1], c[2]);
        const bool xy = tm[0] <= tm[1];
        const int ax = xy ? (tm[0] <= tm[2] ? 0 : 2) : (tm[1] <= tm[2] ? 1 : 2);
        const float tnext = ax == 0 ? tm[0] : (ax == 1 ? tm[1] : tm[2]);
        if (tnext > ry.t1) break;
        if (ax == 0) { c[0] += stp[0]; tm[0] += td[0]; }
        else if (ax == 1) { c[1] += stp[1]; tm[1] += td[1]; }
        else { c[2] += stp[2]; tm[2] += td[2]; }
    }
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
// 1. ray walk and pair emission
// ---------------------------------------------------------------------------

constexpr int kMaxRuns = 8;  // leaf runs per ray; sdf_trunc <= 8 voxel_size keeps a ray within this

__global__ __launch_bounds__(256) void k_ray_walk_emit(FrameParams fp, MapDev md)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    Ray ry;
    bool valid = false;
    if (i < fp.n) {
        const float x = fp.pts[3 * i + 0], y = fp.pts[3 * i + 1], z = fp.pts[3 * i + 2];
        valid = make_ray(fp, x, y, z, ry);
        if (valid && fp.sem_kind == SLIM_IN_LABEL_I32) {
            const int lab = ((const int32_t *)fp.sem)[i];
            valid = lab >= 0 && lab < fp.K;
        }
    }

    // pass 1: count kept cells, check the key range, record the leaf runs
    uint32_t cnt = 0;
    int nruns = 0;
    unsigned long long rkey[kMaxRuns];
    uint32_t rlen[kMaxRuns];
#pragma unroll
    for (int q = 0; q < kMaxRuns; ++q) { rkey[q] = kEmptyKey; rlen[q] = 0; }
    if (valid) {
        bool inrange = true;
        unsigned long long cur = kEmptyKey;
        band_walk(fp, ry, [&](int cx, int cy, int cz) {
            const int kx = fp.a[0] + cx, ky = fp.a[1] + cy, kz = fp.a[2] + cz;
            if (!(key_ok(kx) && key_ok(ky) && key_ok(kz))) { inrange = false; return; }
            if (!(cell_sdf(fp, ry, cx, cy, cz) > -fp.tau)) return;
            const unsigned long long lk = pack_leaf(kx >> 3, ky >> 3, kz >> 3);
            if (lk != cur) {
                cur = lk;
                nruns++;
#pragma unroll
                for (int q = 0; q < kMaxRuns; ++q)
                    if (q == nruns - 1) rkey[q] = lk;
            }
#pragma unroll
            for (int q = 0; q < kMaxRuns; ++q)
                if (q == nruns - 1) rlen[q]++;
            cnt++;
        });
        if (!inrange || nruns > kMaxRuns) valid = false;
    }
    if (!valid) { cnt = 0; nruns = 0; }

    const bool rej = (i < fp.n) && !valid;
    const unsigned long long rejmask = __ballot(rej);
    if (lane_id() == 0 && rejmask) atomicAdd(&md.st->rejected, (unsigned)__popcll(rejmask));

    const uint32_t base = wave_reserve(&md.st->pairs, cnt);

    // stage each run's leaf and reserve its ranks in the leaf's bucket
    uint32_t rpos[kMaxRuns], rrank[kMaxRuns];
#pragma unroll
    for (int q = 0; q < kMaxRuns; ++q) {
        rpos[q] = kNoPos;
        rrank[q] = 0;
        if (q < nruns) {
            const uint32_t pos = stage_leaf(md, rkey[q]);
            rpos[q] = pos;
            if (pos != kNoPos) rrank[q] = atomicAdd(&md.pos_count[pos], rlen[q]);
            else atomicOr(&md.st->frame_err, 1u);
        }
    }
    if (cnt == 0) return;

    // pass 2: write the pairs
    uint32_t o = base, j = 0;
    int run = -1;
    unsigned long long cur = kEmptyKey;
    uint32_t pos = kNoPos, rank = 0;
    band_walk(fp, ry, [&](int cx, int cy, int cz) {
        const float s = cell_sdf(fp, ry, cx, cy, cz);
        if (!(s > -fp.tau)) return;
        const int kx = fp.a[0] + cx, ky = fp.a[1] + cy, kz = fp.a[2] + cz;
        const unsigned long long lk = pack_leaf(kx >> 3, ky >> 3, kz >> 3);
        if (lk != cur) {
            cur = lk;
            run++;
#pragma unroll
            for (int q = 0; q < kMaxRuns; ++q)
                if (q == run) { pos = rpos[q]; rank = rrank[q]; }
        }
        const uint32_t off = (uint32_t)(((kx & 7) << 6) | ((ky & 7) << 3) | (kz & 7));
        if (o + j < md.pair_cap) {
            md.pair_pos[o + j] = pos;
            md.pair_rank[o + j] = rank++;
            md.pair_key[o + j] = (off << kPidBits) | (uint32_t)i;
            md.pair_tsdf[o + j] = fminf(s, fp.tau);
        }
        if (pos != kNoPos) atomicOr(&md.pos_mask[pos * kMaskWords + (off >> 5)], 1u << (off & 31));
        j++;
    });
}

// ---------------------------------------------------------------------------
// 2. leaf planning
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_leaf_plan(MapDev md)
{
    const uint32_t nt = md.st->n_touched;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t jb = blockIdx.x * blockDim.x; jb < nt; jb += stride) {
        const uint32_t j = jb + threadIdx.x;
        const bool act = j < nt;
        int32_t slot = -1;
        uint32_t nnew = 0, nold = 0, npairs = 0, pos = 0;
        if (act) {
            pos = md.touched[j];
            slot = map_find(md, md.skeys[pos]);
            for (int w = 0; w < kMaskWords; ++w) {
                const uint32_t m = md.pos_mask[pos * kMaskWords + w];
                const uint32_t occ = slot >= 0 ? md.leaf_occ[(size_t)slot * kMaskWords + w] : 0u;
                nnew += __popc(m & ~occ);
                nold += __popc(m & occ);
            }
            npairs = md.pos_count[pos];
        }
        const uint32_t newleaf = wave_reserve(&md.st->new_leaves, (act && slot < 0) ? 1u : 0u);
        const uint32_t vbase = wave_reserve(&md.st->new_voxels, nnew);
        const uint32_t bstart = wave_reserve(&md.st->pair_cursor, npairs);
        const uint32_t oldsum = wave_incl_scan(nold);
        if (lane_id() == 63 && oldsum) atomicAdd(&md.st->u_old, (unsigned long long)oldsum);
        if (act) md.pos_plan[pos] = make_int4(slot, slot < 0 ? (int)newleaf : -1, (int)vbase, (int)bstart);
    }
}

// ---------------------------------------------------------------------------
// 3. pair bucketing
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_pair_bucket(MapDev md)
{
    const uint32_t P = min(md.st->pairs, md.pair_cap);
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += stride) {
        const uint32_t pos = md.pair_pos[i];
        if (pos == kNoPos) continue;
        const uint32_t dst = (uint32_t)md.pos_plan[pos].w + md.pair_rank[i];
        md.srt_key[dst] = md.pair_key[i];
        md.srt_tsdf[dst] = md.pair_tsdf[i];
    }
}

// ---------------------------------------------------------------------------
// 4. per-leaf sort, reduce and conjugate combine
// ---------------------------------------------------------------------------

// Ascending sort of n (key, value) pairs by key, in place, by the whole
// workgroup.  Bitonic network in which the first merge step of each stage
// compares mirrored positions, so every block is sorted ascending and
// positions >= n act as +infinity and are never touched.
template <class KP, class VP>
__device__ void block_sort(KP keys, VP vals, uint32_t n)
{
    uint32_t np2 = 1;
    while (np2 < n) np2 <<= 1;
    const uint32_t half = np2 >> 1;
    for (uint32_t k = 2; k <= np2; k <<= 1) {
        // mirrored merge step
        const uint32_t hk = k >> 1;
        for (uint32_t t = threadIdx.x; t < half; t += blockDim.x) {
            const uint32_t blk = t / hk, w = t % hk;
            const uint32_t a = blk * k + w, b = blk * k + k - 1 - w;
            if (b < n) {
                const uint32_t ka = keys[a], kb = keys[b];
                if (kb < ka) {
                    keys[a] = kb; keys[b] = ka;
                    const float va = vals[a];
                    vals[a] = vals[b]; vals[b] = va;
                }
            }
        }
        __syncthreads();
        for (uint32_t d = hk >> 1; d > 0; d >>= 1) {
            for (uint32_t t = threadIdx.x; t < half; t += blockDim.x) {
                const uint32_t a = (t / d) * 2 * d + (t % d), b = a + d;
                if (b < n) {
                    const uint32_t ka = keys[a], kb = keys[b];
                    if (kb < ka) {
                        keys[a] = kb; keys[b] = ka;
                        const float va = vals[a];
                        vals[a] = vals[b]; vals[b] = va;
                    }
                }
            }
            __syncthreads();
        }
    }
}

struct LeafCtx {
    int slot;
    uint32_t n;           // pairs in the bucket
    long long vrec_base;  // first record of this leaf's new voxels
};

// Reduces and combines every voxel segment of a sorted bucket.  G lanes per
// segment; lane r of a group owns semantic components r, r + G, ...
template <int MODE, class KP, class VP>
__device__ void apply_segments(const FrameParams &fp, const MapDev &md, KP keys, VP vals, const LeafCtx &lc,
                               const uint32_t *heads, int nseg, const uint32_t *newmask, const uint32_t *occ0,
                               int G)
{
    const int gid = threadIdx.x / G, lane = threadIdx.x % G, ngroups = blockDim.x / G;
    const size_t lbase = (size_t)lc.slot * kLeafVoxels;
    for (int sg = gid; sg < nseg; sg += ngroups) {
        const uint32_t i0 = heads[sg];
        const uint32_t off = keys[i0] >> kPidBits;
        uint32_t i1 = i0 + 1;
        while (i1 < lc.n && (keys[i1] >> kPidBits) == off) i1++;
        const float nf = (float)(i1 - i0);
        const bool existed = (occ0[off >> 5] >> (off & 31)) & 1u;
        long long rec;
        if (existed) {
            rec = md.leaf_index[lbase + off];
        } else {
            uint32_t rank = 0;
            for (uint32_t w = 0; w < (off >> 5); ++w) rank += __popc(newmask[w]);
            rank += __popc(newmask[off >> 5] & ((1u << (off & 31)) - 1u));
            rec = lc.vrec_base + rank;
            if (lane == 0) md.leaf_index[lbase + off] = (int32_t)rec;
        }
        float2 dw = existed ? md.vox_dw[rec] : make_float2(0.0f, 0.0f);
        const float W0 = dw.y, W1 = W0 + nf;
        if (lane == 0) {
            // Eq. (1)-(2), unit weights: D' = (W D + sum tsdf) / (W + n)
            float st = 0.0f;
            for (uint32_t i = i0; i < i1; ++i) st += vals[i];
            md.vox_dw[rec] = make_float2((W0 * dw.x + st) / W1, W1);
        }
        if (MODE == SLIM_SEM_CLOSED) {
            float *S = md.vox_sem + (size_t)rec * fp.nsem;
            if (fp.sem_kind == SLIM_IN_LOGIT_F32) {
                // K <= G: lane k owns class k; softmax per observation across the group
                const float *lg = (const float *)fp.sem;
                float acc = 0.0f;
                for (uint32_t i = i0; i < i1; ++i) {
                    const uint32_t pid = keys[i] & kPidMask;
                    const float l = lane < fp.K ? lg[(size_t)pid * fp.K + lane] : -INFINITY;
                    float mx = l;
                    for (int d = G >> 1; d > 0; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d, G));
                    const float e = lane < fp.K ? expf(l - mx) : 0.0f;
                    float den = e;
                    for (int d = G >> 1; d > 0; d >>= 1) den += __shfl_xor(den, d, G);
                    acc += e / den;
                }
                if (lane < fp.K) S[lane] = (existed ? S[lane] : 0.0f) + acc;
            } else {
                for (int k = lane; k < fp.K; k += G) {
                    float acc = 0.0f;
                    if (fp.sem_kind == SLIM_IN_LABEL_I32) {
                        const int32_t *lb = (const int32_t *)fp.sem;
                        for (uint32_t i = i0; i < i1; ++i) acc += (lb[keys[i] & kPidMask] == k) ? 1.0f : 0.0f;
                    } else {
                        const float *pr = (const float *)fp.sem;
                        for (uint32_t i = i0; i < i1; ++i) acc += pr[(size_t)(keys[i] & kPidMask) * fp.K + k];
                    }
                    // Eq. (6): concentrations grow by the (expected) counts
                    S[k] = (existed ? S[k] : 0.0f) + acc;
                }
            }
        } else if (MODE == SLIM_SEM_OPEN) {
            float *M = md.vox_sem + (size_t)rec * fp.nsem;
            float *B = M + fp.L;
            const bool bf = fp.sem_kind == SLIM_IN_EMB_BF16;
            const float inv_n = 1.0f / nf;
            const float cross = W0 * nf / W1;
            for (int d = lane; d < fp.L; d += G) {
                float s1 = 0.0f;
                for (uint32_t i = i0; i < i1; ++i) {
                    const size_t idx = (size_t)(keys[i] & kPidMask) * fp.L + d;
                    s1 += bf ? __uint_as_float((uint32_t)((const uint16_t *)fp.sem)[idx] << 16)
                             : ((const float *)fp.sem)[idx];
                }
                const float zbar = s1 * inv_n;
                float s2 = 0.0f;
                for (uint32_t i = i0; i < i1; ++i) {
                    const size_t idx = (size_t)(keys[i] & kPidMask) * fp.L + d;
                    const float z = bf ? __uint_as_float((uint32_t)((const uint16_t *)fp.sem)[idx] << 16)
                                       : ((const float *)fp.sem)[idx];
                    const float dz = z - zbar;
                    s2 += dz * dz;
                }
                // Eqs. (11)-(14) with lambda = W, nu = W / 2
                const float m0 = existed ? M[d] : 0.0f, b0 = existed ? B[d] : 0.0f;
                const float dm = zbar - m0;
                B[d] = b0 + 0.5f * s2 + cross * dm * dm * 0.5f;
                M[d] = (W0 * m0 + nf * zbar) / W1;
            }
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(kApplyThreads) void k_leaf_apply(FrameParams fp, MapDev md, int G)
{
    __shared__ uint32_t s_key[kApplyLdsPairs];
    __shared__ float s_val[kApplyLdsPairs];
    __shared__ uint32_t s_heads[kLeafVoxels];
    __shared__ uint32_t s_newmask[kMaskWords], s_occ0[kMaskWords];
    __shared__ int s_nseg, s_slot, s_last;

    DevState *st = md.st;
    const uint32_t nt = st->n_touched;
    const unsigned long long lused = st->leaves_used, vused = st->voxels_used;
    const unsigned long long nl = st->new_leaves, nv = st->new_voxels;
    const bool ok = st->frame_err == 0 && lused + nl <= (unsigned long long)md.max_leaves &&
                    vused + nv <= (unsigned long long)md.max_voxels;

    for (uint32_t j = blockIdx.x; j < nt; j += gridDim.x) {
        const uint32_t pos = md.touched[j];
        const int4 plan = md.pos_plan[pos];
        const uint32_t n = md.pos_count[pos];
        if (ok) {
            if (threadIdx.x == 0) {
                int slot = plan.x;
                if (slot < 0) {
                    slot = (int)(lused + (unsigned long long)plan.y);
                    const unsigned long long key = md.skeys[pos];
                    map_insert(md, key, slot);
                    md.leaf_key[slot] = key;
                }
                s_slot = slot;
                s_nseg = 0;
            }
            __syncthreads();
            const int slot = s_slot;
            if (plan.x < 0)
                for (int t = threadIdx.x; t < kLeafVoxels; t += blockDim.x)
                    md.leaf_index[(size_t)slot * kLeafVoxels + t] = -1;
            if (threadIdx.x < kMaskWords) {
                const uint32_t occ = plan.x < 0 ? 0u : md.leaf_occ[(size_t)slot * kMaskWords + threadIdx.x];
                const uint32_t m = md.pos_mask[(size_t)pos * kMaskWords + threadIdx.x];
                s_occ0[threadIdx.x] = occ;
                s_newmask[threadIdx.x] = m & ~occ;
            }
            LeafCtx lc;
            lc.slot = slot;
            lc.n = n;
            lc.vrec_base = (long long)vused + plan.z;
            uint32_t *gk = md.srt_key + plan.w;
            float *gv = md.srt_tsdf + plan.w;
            if (n <= (uint32_t)kApplyLdsPairs) {
                for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) {
                    s_key[t] = gk[t];
                    s_val[t] = gv[t];
                }
                __syncthreads();
                block_sort(s_key, s_val, n);
                for (uint32_t t = threadIdx.x; t < n; t += blockDim.x)
                    if (t == 0 || (s_key[t] >> kPidBits) != (s_key[t - 1] >> kPidBits))
                        s_heads[atomicAdd(&s_nseg, 1)] = t;
                __syncthreads();
                apply_segments<MODE>(fp, md, s_key, s_val, lc, s_heads, s_nseg, s_newmask, s_occ0, G);
            } else {
                __syncthreads();
                block_sort(gk, gv, n);
                for (uint32_t t = threadIdx.x; t < n; t += blockDim.x)
                    if (t == 0 || (gk[t] >> kPidBits) != (gk[t - 1] >> kPidBits))
                        s_heads[atomicAdd(&s_nseg, 1)] = t;
                __syncthreads();
                apply_segments<MODE>(fp, md, gk, gv, lc, s_heads, s_nseg, s_newmask, s_occ0, G);
            }
            if (threadIdx.x < kMaskWords)
                md.leaf_occ[(size_t)slot * kMaskWords + threadIdx.x] = s_occ0[threadIdx.x] | s_newmask[threadIdx.x];
        }
        // the staging entry of this leaf is clean for the next frame
        if (threadIdx.x < kMaskWords) md.pos_mask[(size_t)pos * kMaskWords + threadIdx.x] = 0u;
        if (threadIdx.x == 0) {
            md.pos_count[pos] = 0u;
            md.skeys[pos] = kEmptyKey;
        }
        __syncthreads();
    }

    // the last workgroup commits the frame and clears the frame counters
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(&st->done_blocks, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        const int err = st->frame_err ? SLIM_ERR_CAPACITY : (ok ? SLIM_OK : SLIM_ERR_CAPACITY);
        if (err == SLIM_OK) {
            st->leaves_used = lused + nl;
            st->voxels_used = vused + nv;
        } else if (st->status == SLIM_OK) {
            st->status = err;
        }
        st->last_points = fp.n;
        st->last_rejected = st->rejected;
        st->last_pairs = st->pairs;
        st->last_touched = nt;
        st->last_new_leaves = nl;
        st->last_u_old = (long long)st->u_old;
        st->last_u_new = nv;
        st->last_status = err;
        st->n_touched = 0;
        st->pairs = 0;
        st->rejected = 0;
        st->new_leaves = 0;
        st->new_voxels = 0;
        st->pair_cursor = 0;
        st->u_old = 0;
        st->frame_err = 0;
        __threadfence();
        st->done_blocks = 0;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_integrate(const FrameParams &fp, const MapDev &md, int apply_blocks, hipStream_t s,
                            hipEvent_t *ev)
{
    const int bw = (fp.n + 255) / 256;
    auto rec = [&](int e) {
        if (ev) (void)hipEventRecord(ev[e], s);
    };
    rec(0);
    hipLaunchKernelGGL(k_ray_walk_emit, dim3(bw > 0 ? bw : 1), dim3(256), 0, s, fp, md);
    rec(1);
    rec(2);
    hipLaunchKernelGGL(k_leaf_plan, dim3(256), dim3(256), 0, s, md);
    rec(3);
    rec(4);
    hipLaunchKernelGGL(k_pair_bucket, dim3(1024), dim3(256), 0, s, md);
    rec(5);
    int G = 1;
    if (fp.sem_kind != SLIM_IN_NONE) {
        const int want = (fp.nsem == 0) ? 1 : (fp.L > 0 ? 64 : fp.K);
        while (G < want && G < 64) G <<= 1;
    }
    rec(6);
    if (fp.L > 0)
        hipLaunchKernelGGL(k_leaf_apply<SLIM_SEM_OPEN>, dim3(apply_blocks), dim3(kApplyThreads), 0, s, fp, md, G);
    else if (fp.K > 0)
        hipLaunchKernelGGL(k_leaf_apply<SLIM_SEM_CLOSED>, dim3(apply_blocks), dim3(kApplyThreads), 0, s, fp, md, G);
    else
        hipLaunchKernelGGL(k_leaf_apply<SLIM_SEM_NONE>, dim3(apply_blocks), dim3(kApplyThreads), 0, s, fp, md, G);
    rec(7);
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

__global__ void k_reset_state(DevState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        DevState z = {};
        *st = z;
    }
}

hipError_t launch_reset(const MapDev &md, hipStream_t s)
{
    const size_t cap = (size_t)md.hmask + 1;
    hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, md.hkeys, cap, kEmptyKey);
    hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, md.skeys, cap, kEmptyKey);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, md.pos_count, cap, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, md.pos_mask, cap * kMaskWords, 0u);
    hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, md.st);
    return hipGetLastError();
}

__global__ void k_collect_leaves(const MapDev md, long long nleaves, unsigned long long *keys, int32_t *slots)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nleaves;
         i += (long long)gridDim.x * blockDim.x) {
        keys[i] = md.leaf_key[i];
        slots[i] = (int32_t)i;
    }
}

// One compare-exchange step of the mirrored bitonic network over n elements
// (virtual +infinity beyond n), in global memory.
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
            uint32_t rank = 0;
            for (int q = 0; q < (t >> 5); ++q) rank += __popc(occ[q]);
            rank += __popc(occ[t >> 5] & ((1u << (t & 31)) - 1u));
            const size_t o = (size_t)offsets[j] + rank;
            const long long rec = md.leaf_index[(size_t)slot * kLeafVoxels + t];
            keys[3 * o + 0] = lx * 8 + (t >> 6);
            keys[3 * o + 1] = ly * 8 + ((t >> 3) & 7);
            keys[3 * o + 2] = lz * 8 + (t & 7);
            const float2 dw = md.vox_dw[rec];
            d[o] = dw.x;
            w[o] = dw.y;
            if (sem)
                for (int k = 0; k < nsem; ++k) sem[o * nsem + k] = md.vox_sem[(size_t)rec * nsem + k];
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

__global__ __launch_bounds__(256) void k_query(const MapDev md, int nsem, float vs, const float *xyz, long long m,
                                               float *d, float *w, float *sem)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x) {
        long long rec = -1;
        const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (isfinite(x) && isfinite(y) && isfinite(z)) {
            const float fx = floorf(x / vs), fy = floorf(y / vs), fz = floorf(z / vs);
            const float lim = (float)kKeyLimit;
            if (fabsf(fx) < lim && fabsf(fy) < lim && fabsf(fz) < lim) {
                const int kx = (int)fx, ky = (int)fy, kz = (int)fz;
                const int slot = map_find(md, pack_leaf(kx >> 3, ky >> 3, kz >> 3));
                if (slot >= 0) {
                    const int off = ((kx & 7) << 6) | ((ky & 7) << 3) | (kz & 7);
                    if ((md.leaf_occ[(size_t)slot * kMaskWords + (off >> 5)] >> (off & 31)) & 1u)
                        rec = md.leaf_index[(size_t)slot * kLeafVoxels + off];
                }
            }
        }
        if (rec >= 0) {
            const float2 dw = md.vox_dw[rec];
            d[i] = dw.x;
            w[i] = dw.y;
            if (sem)
                for (int k = 0; k < nsem; ++k) sem[i * nsem + k] = md.vox_sem[(size_t)rec * nsem + k];
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

}  // namespace slim
