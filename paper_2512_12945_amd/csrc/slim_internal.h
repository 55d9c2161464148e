// Internal types shared by the host runtime and the kernels of libslimvdb.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slim {

constexpr uint64_t kEmptyKey = ~0ull;        // free slot of a leaf table
constexpr uint32_t kNoPos = 0xFFFFFFFFu;     // pair whose leaf could not be staged
constexpr int kKeyLimit = 1 << 20;           // voxel coordinates satisfy |k| < 2^20
constexpr int kLeafBias = 1 << 17;           // leaf coordinates, biased into 18 bits
constexpr int kPidBits = 23;                 // point index bits of a sort key
constexpr uint32_t kPidMask = (1u << kPidBits) - 1u;
constexpr int64_t kMaxPoints = int64_t(1) << kPidBits;
constexpr int kLeafVoxels = 512;
constexpr int kMaskWords = kLeafVoxels / 32; // 16 words of touched/occupied bits per leaf
constexpr int kSortThreads = 256;
constexpr int kSortBatch = 8;                // loads in flight per thread in the leaf sort
constexpr int kSortLdsPairs = kSortBatch * kSortThreads;  // a leaf's pairs sort in LDS up to this many
constexpr uint32_t kSegChunk = 64;           // segment-to-leaf lookup marks every this many segments
constexpr int kNumProfiled = 6;
constexpr int kWalkThreads = 256;
constexpr int kWalkTable = 2048;             // block-local leaf table of the walk kernel

// segment descriptor meta bits
constexpr uint32_t kSegOffMask = 0x1FFu;     // voxel offset in its leaf
constexpr uint32_t kSegExisted = 1u << 9;    // voxel had a record before this frame
constexpr uint32_t kSegFirst = 1u << 10;     // first segment (lowest offset) of its leaf

// floats of one voxel record: D, W, then the semantic state, padded to 16 bytes
__host__ __device__ inline int record_stride(int nsem) { return (2 + nsem + 3) & ~3; }

// Device-resident counters of one map.  Counters that many blocks update sit
// on cache lines of their own (same-line atomics serialise).  Frame counters
// are zero between frames: the allocation kernel snapshots and clears them.
struct alignas(128) Line {
    unsigned int v;
    unsigned int pad[31];
};

struct ApplyParams {           // what the apply kernel needs, fixed by the allocation kernel
    unsigned int nt;           // leaves touched
    unsigned int nseg;         // voxels touched
    unsigned int ok;           // frame fits: apply it
    unsigned int pad;
    unsigned long long lused0; // leaves before the frame
    unsigned long long vused0; // voxel records before the frame
};

struct DevState {
    // hot frame counters
    Line pairs;       // (voxel, point) observations emitted
    Line n_touched;   // leaves touched (staging-table entries)
    Line rejected;    // points rejected
    Line new_leaves;  // leaves to create
    Line pair_cursor; // bucket allocation cursor
    Line frame_err;   // nonzero: do not apply this frame
    // persistent
    unsigned long long leaves_used;
    unsigned long long voxels_used;
    int status;       // first asynchronous error not yet reported
    int pad0;
    ApplyParams ap;
    // last frame (written by the allocation kernel)
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
    const float *pts;  // n x 3
    const void *sem;   // per-point semantics
};

// Device pointers of one map.
struct MapDev {
    // leaf table: packed leaf key -> leaf slot, open addressing, cap = hmask + 1
    unsigned long long *hkeys;
    int32_t *hvals;
    // staging table of the leaves one frame touches (same capacity)
    unsigned long long *skeys;
    uint32_t *touched;   // staging positions in insertion order
    uint32_t *pos_count; // pairs per staging position
    uint32_t *pos_occ;   // 16 words per position: the leaf's occupancy after this frame
    int4 *pos_plan;      // (slot or -1, new-leaf index, bucket start, 0)
    uint2 *leaf_cnt;     // per touched-list index: (voxels touched, voxels created)
    uint2 *leaf_base;    // per touched-list index: exclusive sums of leaf_cnt
    int4 *leaf_info;     // per touched-list index: (bucket start, slot or -1 - new-leaf index, staging position, 0)
    uint32_t *chunk_leaf;// leaf (touched-list index) of segments 0, kSegChunk, 2 kSegChunk, ...
    uint32_t hmask;
    // leaves
    unsigned long long *leaf_key; // packed key per slot
    int32_t *leaf_index;          // 512 voxel record indices per slot (-1: none)
    uint32_t *leaf_occ;           // 16 words per slot: offsets with a record
    // voxel records: record_stride(nsem) floats each, D, W, then semantics
    float *vox;
    int rec_stride;
    // per-frame pair buffers
    uint32_t *pair_pos;   // staging position of the pair's leaf
    uint32_t *pair_rank;  // rank of the pair inside its leaf's bucket
    uint32_t *pair_key;   // (offset << 23) | point index
    float *pair_tsdf;     // truncated signed distance (FP32)
    uint32_t *srt_key;    // pairs grouped by leaf, then sorted by (offset, point)
    float *srt_tsdf;
    uint32_t *tmp_key;    // scratch of the in-memory sort of large leaves
    float *tmp_tsdf;
    int4 *seg_desc;       // per touched voxel, at (bucket start + voxel rank in its leaf):
                          // (first pair, pair count, record or new-voxel rank, meta bits)
    uint32_t pair_cap;
    DevState *st;
    long long max_leaves, max_voxels;
};

__host__ __device__ inline unsigned long long pack_leaf(int lx, int ly, int lz)
{
    return ((unsigned long long)(uint32_t)(lx + kLeafBias) << 36) |
           ((unsigned long long)(uint32_t)(ly + kLeafBias) << 18) |
           (unsigned long long)(uint32_t)(lz + kLeafBias);
}

// kernel launchers (slimvdb_kernels.hip)
hipError_t launch_integrate(const FrameParams &fp, const MapDev &md, int cus, hipStream_t s,
                            hipEvent_t *ev /* 2 * kNumProfiled events or nullptr */);
hipError_t launch_reset(const MapDev &md, hipStream_t s);
hipError_t launch_extract(const MapDev &md, int nsem, long long nleaves, unsigned long long *tmp_keys,
                          int32_t *tmp_slots, uint32_t *tmp_offsets, int32_t *keys, float *d, float *w, float *sem,
                          hipStream_t s);
hipError_t launch_query(const MapDev &md, int nsem, float vs, const float *xyz, long long m, float *d, float *w,
                        float *sem, hipStream_t s);

}  // namespace slim
