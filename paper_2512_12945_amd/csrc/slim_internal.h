// Internal types shared by the host runtime and the kernels of libslimvdb.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "slimvdb.h"

namespace slim {

constexpr uint64_t kEmptyKey = ~0ull;        // free slot of a leaf table
constexpr uint32_t kNoPos = 0xFFFFFFFFu;     // pair whose leaf could not be staged
constexpr int kKeyLimit = 1 << 20;           // voxel coordinates satisfy |k| < 2^20
constexpr int kLeafBias = 1 << 17;           // leaf coordinates, biased into 18 bits
constexpr int kPidBits = 23;                 // point index bits of a sort key
constexpr uint32_t kPidMask = (1u << kPidBits) - 1u;
constexpr int64_t kMaxPoints = int64_t(1) << kPidBits;
constexpr int kLeafVoxels = 512;
constexpr int kMaskWords = kLeafVoxels / 32; // 16 words of occupied bits per leaf
constexpr int kPageVoxels = 64;              // records are allocated per x-slab (8 x 8 voxels) of a leaf
constexpr int kLeafPages = kLeafVoxels / kPageVoxels;
#ifndef SLIM_WALK_THREADS
#define SLIM_WALK_THREADS 256
#endif
constexpr int kWalkThreads = SLIM_WALK_THREADS;  // rays per walk block
constexpr int kWalkTable = 8 * kWalkThreads;     // block-local leaf table: at most 8 leaf runs per ray
constexpr int kLeafThreads = 256;
constexpr int kLeafBatch = 8;                // loads in flight per thread in the leaf kernel
constexpr int kLeafLdsPairs = kLeafBatch * kLeafThreads;  // pairs a leaf holds in LDS at once
constexpr int kNumProfiled = 6;  // timed stages: walk, plan, bucketing, leaf kernel, voxel combine, commit
constexpr int kAccFrames = 8;        // frames of a pass the accumulating leaf kernel takes
constexpr int kAccWavePairs = 128;   // accumulated leaves with at most this many pairs are one wave's work
constexpr int kPassFrames = 8;               // most frames integrated in one pass
constexpr int kMaxLeafBlocksPerCu = 32;

// floats of one voxel record: D, W, then the semantic state, padded to 16 bytes
__host__ __device__ inline int record_stride(int nsem) { return (2 + nsem + 3) & ~3; }

// Counters that many blocks update sit on cache lines of their own (same-line
// atomics serialise).
struct alignas(128) Line {
    unsigned int v;
    unsigned int pad[31];
};

// Counters of the frame in flight on one staging buffer.  They are zero
// between frames: the commit kernel clears them.
struct FrameState {
    Line pairs;       // (voxel, point) observations emitted
    Line n_touched;   // leaves touched (staging-table entries)
    Line rejected;    // points rejected
    Line new_leaves;  // leaves to create
    Line new_pages;   // record pages to create
    Line pair_cursor; // bucket allocation cursor
    Line work_big;    // slab work items of large leaves
    // leaves done by one workgroup (low half) and by one wave (high half): the
    // larger ones of each list from the front of its array, the smaller ones
    // from the back, so that the leaf kernel starts the longer work first
    alignas(128) unsigned long long n_lists;
    unsigned int pad_lists[30];
    alignas(128) unsigned long long n_lists_tail;
    unsigned int pad_tail[30];
    Line n_vox;       // voxel descriptors for the wave combine
    Line frame_err;   // nonzero: do not apply this frame
};

// Device-resident counters of one map.
struct DevState {
    unsigned long long leaves_used;
    unsigned long long pages_used;
    unsigned long long voxels_used;  // voxels with W > 0
    int status;       // first asynchronous error not yet reported
    int pass_failed;  // 0, or 1 + the first frame of a multi-frame pass that could not be applied
    // last frame (written by the commit)
    long long last_points, last_rejected, last_pairs, last_touched, last_new_leaves, last_u_old, last_u_new;
    int last_status;
    int pad1;
};

// Geometry of one frame, canonicalised on the host (FP64 -> FP32).
struct FrameParams {
    float R[9];        // rotation of map_T_sensor, rounded to binary32
    float t[3];        // sensor origin relative to the anchor voxel's corner
    int a[3];          // anchor voxel (holds the sensor origin)
    float vs, tau, rmin, rmax;
    int maxsteps;      // cap on voxels visited per ray
    int n;             // points
    int sem_kind;      // SLIM_IN_*
    int K, L, nsem;    // classes, embedding dim, floats of semantic state per voxel
    int last;          // 1: non-Bayesian mode, a voxel keeps its most recent measurement
    const float *pts;  // n x 3, or NULL when the points come as ranges and directions
    const float *ranges, *dirs;  // n and n x 3: point = range * direction
    const float *depth;          // or a row-major depth image, n = width * height pixels
    int width;
    float fx, fy, cx, cy;        // pinhole intrinsics of the depth image
    const void *sem;   // per-point semantics
    // several consecutive frames integrated in one pass: every frame's point
    // indices are offset so that they are distinct across the pass
    uint32_t pid_base;                  // offset of this frame's point indices
    int nsub;                           // frames of the pass (0 or 1: a frame on its own)
    int pass_first;                     // the pass's first frame in its sequence call
    uint32_t sub_start[kPassFrames + 1];  // offset of each frame of the pass, then the pass's total
    const void *sub_sem[kPassFrames];     // per-point semantics of each frame of the pass
};

// Frames whose voxels only gain integers (counts, class counts of int32 labels
// with K <= 32, fixed-point distance sums): their leaves are accumulated in any
// order, without sorting, and several such frames can share one pass.
__host__ __device__ inline bool accum_path(const FrameParams &fp)
{
    if (fp.last || fp.L > 0) return false;
    return fp.K == 0 || (fp.K <= 32 && fp.sem_kind == SLIM_IN_LABEL_I32);
}

// The walk of a multi-frame pass: each frame's rays, one block range per frame.
struct PassWalk {
    FrameParams fp[kPassFrames];
    int blk_start[kPassFrames + 1];
    int nframes;
};
static_assert(sizeof(PassWalk) + 512 <= 4096, "the pass walk's kernel arguments fit the 4 KiB argument buffer");

// Inputs and outputs of the map loss and its backward.
struct LossParams {
    const int32_t *keys;     // m x 3 voxel keys (all voxels of the map)
    const int32_t *labels;   // m ground-truth classes
    long long m;
    const float *samples;    // s x 3 world points
    long long s;
    float alpha0;
    float *loss;             // 3 floats: total, cross-entropy term, L1 term
    float *adj;              // per record: K adjoints dL/dc, then dL/dD (stride adj_stride)
    int32_t *adj_cnt;        // per record: surface samples in the voxel
    int adj_stride;
    float *part;             // block partial sums
    int32_t *part_cnt;       // block partial sample counts
};

// Everything the leaf kernel needs of one touched leaf, written by the plan
// kernel where the leaf kernel's unit of work finds it (see MapDev::items), so
// that one 128-byte read starts its work.
struct alignas(16) LeafItem {
    uint32_t pos;             // staging position
    uint32_t n;               // pairs
    uint32_t bstart;          // first pair of its bucket
    int32_t slot;             // leaf slot, or -1 - (index among this frame's new leaves)
    uint32_t slabs;           // x-slabs touched this frame (8 bits)
    uint32_t pad;
    unsigned long long key;   // packed leaf key
    int32_t pages[8];         // record page of each slab (-1: none)
    uint32_t occ[16];         // voxels with W > 0 before this frame
};
static_assert(sizeof(LeafItem) == 128, "a leaf item is 128 bytes");

// One slot of the leaf table: packed leaf key (kEmptyKey: free) and leaf
// slot, read together with one 16-byte load.
struct alignas(16) HashSlot {
    unsigned long long key;
    int32_t val;
    int32_t pad;
};

// Device pointers of one map.
struct MapDev {
    // leaf table: packed leaf key -> leaf slot, open addressing, cap = hmask + 1
    HashSlot *htab;
    uint32_t hmask;
    // staging table of the leaves one frame touches (same capacity), and
    // per-position frame data
    unsigned long long *skeys;
    uint32_t *touched;   // staging positions in insertion order
    unsigned long long *touched_key;  // their packed leaf keys
    uint32_t *pos_count; // pairs per position
    uint32_t *pos_slab;  // x-slabs of the leaf the frame touches (8 bits)
    int4 *pos_plan;      // (slot or -1, new-leaf index, bucket start, 0)
    int4 *pos_pages;     // 2 per position: record page of each of the 8 slabs (-1: none)
    // the leaf kernel's view of each touched leaf, written by the plan kernel
    // where the leaf kernel's unit finds it without another lookup: leaves done
    // by one workgroup and by one wave in the order of their work lists (the
    // larger ones from the front of the array, the smaller ones from the back),
    // large leaves at the index of their first slab work item
    LeafItem *items;       // leaves done by one workgroup (cap entries)
    LeafItem *items_small; // leaves done by one wave (cap entries)
    LeafItem *items_big;   // large leaves (work_cap entries)
    // leaves
    unsigned long long *leaf_key; // packed key per slot
    int32_t *leaf_page;           // 8 record pages per slot (-1: none)
    uint32_t *leaf_occ;           // 16 words per slot: voxels with W > 0
    // voxel records: page p holds records 64 p .. 64 p + 63 (slab offset y * 8 + z),
    // record_stride(nsem) floats each: D, W, then semantics
    float *vox;
    int rec_stride;
    // per-frame pair buffers
    uint4 *pairs;         // the walk's pairs: (staging position of the pair's leaf, rank of the pair
                          // inside its leaf's bucket, (offset << 23) | point index, truncated distance bits)
    uint32_t *pair_key;   // leaf-kernel scratch: sorted keys of bins beyond LDS, wave-combine input
    float *pair_tsdf;     // and their truncated distances
    uint2 *srt_kv;        // pairs grouped by leaf: (key, truncated distance bits)
    int32_t *srt_lab;     // int32 label of each bucketed pair (closed set with labels)
    uint32_t *tmp_key;    // scratch of large leaves: pairs binned by voxel offset
    float *tmp_tsdf;
    uint32_t pair_cap;
    int2 *work;           // slab work items (index in items_big, slab) of large leaves
    uint32_t work_cap;
    uint4 *vox_list;      // wave-combine voxels: (record, pairs | existed << 31, first sorted pair, 0)
    uint2 *blk_stats;     // per leaf-kernel block: (voxels updated that existed, voxels created)
    int leaf_blocks;      // grid of the leaf kernel of the current frame (<= kMaxLeafBlocksPerCu * CUs)
    // leaf tiles of the current frame: leaves with at most wave_pairs pairs are
    // one wave's work, sorted leaves with more than slab_pairs pairs are split
    // into x-slab items (0: the largest the kernels hold)
    int wave_pairs, slab_pairs;
    DevState *st;
    FrameState *fs;       // the staging buffer's frame counters
    long long max_leaves, max_pages;
};

// Device descriptor of a batched launch over several maps (one frame each).
// Each per-stage launch is shared between its maps: map q of the launch holds
// blocks first[q] .. first[q + 1] - 1 and runs the stage's grid-stride code
// with that share as its grid.
struct MapBatch {
    const MapDev *mds;       // nmaps
    const FrameParams *fps;  // nmaps
    const int *walk_start;   // nmaps + 1: first walk block of each map
    const int *subset;       // the maps one leaf-kernel launch handles
    const int *plan_first, *bucket_first;  // nmaps + 1 each
    const int *part_first;   // nsubset + 1: the shares of a leaf-kernel or combine launch
    int nmaps, nsubset;
};

// Grid sizes of the grid-stride kernels, and the work split of the persistent
// batched launch (results do not depend on any of them).
struct LaunchShape {
    int plan_blocks;    // leaf planning
    int bucket_blocks;  // pair bucketing
    int leaf_blocks;    // per-leaf sort and combine (also the size of blk_stats in use)
    int persistent;     // batched calls: 1 one persistent launch, 0 one launch per stage
    int walk_chunk;     // persistent: walk blocks (256 rays each) per ray-chunk item
    int wave_pairs;     // leaf tiles (MapDev::wave_pairs, slab_pairs)
    int slab_pairs;
    int cus;            // compute units of the map's GPU
};

// Host view of a batched launch: the leaf kernel is launched once per group of
// maps that share its template (classes in registers, wave per voxel, rows).
struct BatchPlan {
    int nmaps;
    int walk_blocks;                 // total blocks of the walk kernel
    int plan_blocks, bucket_blocks;  // grids of planning and bucketing
    int ngroups;
    int group_kind[17];                   // leaf-kernel variant of each group
    int group_begin[17], group_size[17];  // slice of the device subset array
    int leaf_blocks[17], comb_blocks[17]; // grids of each group's leaf-kernel and combine launches
    int leaf_part[17], comb_part[17];     // offsets of their shares in the device share arrays
};

constexpr int kLeafKinds = 17;  // variants of the leaf kernel (leaf_kernel_kind)
int leaf_kernel_kind(const FrameParams &fp);
__host__ __device__ int voxel_combine_arg(int kind);
int combine_blocks(int kind, const LaunchShape &shape);
hipError_t launch_integrate_batched(const MapBatch &mb, const BatchPlan &plan, const LaunchShape &shape,
                                    hipStream_t s);

// Persistent batched launch: work items (uint4) taken from a queue in order,
//   x = map | stage << 16 | leaf-kernel variant << 24,
//   y, z = first walk block and walk blocks (stage 0), or item index and items
//          of the stage for the map (grid-stride stages),
//   w = the counter to wait for | its target << 16, or kPersistNoDep;
// and a control block of uint32 words, zero at launch:
//   [0] next item, [1] abort flag, [2 + map * kPersistStages + stage] finished items.
constexpr int kPersistStages = 6;  // walk, planning, bucketing, leaf kernel, voxel combine, commit
constexpr uint32_t kPersistEnd = 0xFFFFFFFFu;
constexpr uint32_t kPersistNoDep = 0xFFFFFFFFu;
constexpr int kPersistCtlAbort = 1;
constexpr int kPersistCtlDone = 2;
struct PersistArgs {
    const MapDev *mds;
    const FrameParams *fps;
    const uint4 *items;
    uint32_t *ctl;
    uint32_t nitems;
};
int persistent_blocks_per_cu();
hipError_t launch_integrate_persistent(const PersistArgs &a, int blocks, hipStream_t s);

__host__ __device__ inline unsigned long long pack_leaf(int lx, int ly, int lz)
{
    return ((unsigned long long)(uint32_t)(lx + kLeafBias) << 36) |
           ((unsigned long long)(uint32_t)(ly + kLeafBias) << 18) |
           (unsigned long long)(uint32_t)(lz + kLeafBias);
}

// kernel launchers (slimvdb_kernels.hip)
hipError_t launch_integrate(const FrameParams &fp, const MapDev &md, const LaunchShape &shape, hipStream_t s,
                            hipEvent_t *ev /* 2 * kNumProfiled events or nullptr */,
                            const PassWalk *pw = nullptr /* the walk of a multi-frame pass */);
hipError_t launch_reset(const MapDev &md, hipStream_t s);
hipError_t launch_reset_staging(const MapDev &md, hipStream_t s);
hipError_t launch_walk(const FrameParams &fp, const MapDev &md, hipStream_t s, const PassWalk *pw = nullptr);
hipError_t launch_after_walk(const FrameParams &fp, const MapDev &md, const LaunchShape &shape, hipStream_t s);
hipError_t launch_loss(const FrameParams &fp, const MapDev &md, const LossParams &lp, hipStream_t s);
hipError_t launch_backward(const FrameParams &fp, const MapDev &md, const LossParams &lp, const float *grad_scale,
                           float *grad_logits, float *grad_ranges, hipStream_t s);
constexpr int kLossThreads = 256;
hipError_t launch_extract(const MapDev &md, int nsem, long long nleaves, unsigned long long *tmp_keys,
                          int32_t *tmp_slots, uint32_t *tmp_offsets, int32_t *keys, float *d, float *w, float *sem,
                          hipStream_t s);
// Allocation-free extract: its per-leaf scratch (key 8 B, slot 4 B, voxel
// offset 4 B) lives in a file-scope device array of the library, one copy per
// GPU, for at most kNoAllocMaxLeaves leaves.
constexpr long long kNoAllocMaxLeaves = 1ll << 20;
constexpr int kNoAllocMaxDevices = 64;
// With the device current, resolves that GPU's address of the array (once per
// device; later calls return at once).
hipError_t noalloc_scratch_setup(int device);
// The address resolved for `device`, or nullptr if setup has not succeeded.
void *noalloc_scratch(int device);
// Semantic read-out (slim_predict).
struct PredictParams {
    float vs, alpha0, inv_temp, threshold;
    int mode;               // SLIM_SEM_*
    int K, L, P;            // classes, embedding dim, prototypes
    const float *protos;    // P x L
};
hipError_t launch_predict(const MapDev &md, const PredictParams &pp, const float *xyz, long long m, float *prob,
                          int32_t *label, float *var, hipStream_t s);
// Render of the map from a pinhole camera (slim_render).
struct RenderParams {
    float R[9], t[3];      // camera rotation (binary32) and origin relative to the anchor voxel's corner
    int a[3];              // anchor voxel
    float vs, fx, fy, cx, cy, t0, t1;
    int maxsteps, width, height;
    int mode, K;           // SLIM_SEM_* and classes, for the label
};
hipError_t launch_render(const MapDev &md, const RenderParams &rp, float *depth, int32_t *key, int32_t *label,
                         hipStream_t s);
hipError_t launch_query(const MapDev &md, int nsem, float vs, const float *xyz, long long m, float *d, float *w,
                        float *sem, hipStream_t s);

}  // namespace slim
