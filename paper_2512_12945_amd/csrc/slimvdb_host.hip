// Host runtime and C ABI of the semantic TSDF integrator: validation, map
// memory, pose canonicalisation, launches, read-back and kernel timing.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "slim_internal.h"
#include "slimvdb.h"

using namespace slim;

namespace {

thread_local char g_err[512] = "";

slim_status fail(slim_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_OK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(SLIM_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev_ >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
    }

  private:
    int prev_ = -1;
};

constexpr int kProfRing = 256;  // frames whose kernel events may be outstanding
constexpr size_t kMaxProfSets = 1 << 16;  // launch sets kept for slim_profile_sets

}  // namespace

// Launch resources of batched integration, owned by the first map of a batch.
struct BatchCtx {
    void *staging = nullptr;  // pinned host copy of the descriptor
    void *dev = nullptr;      // device descriptor
    size_t cap = 0;
    hipEvent_t copied = nullptr;  // staging may be rewritten once this has fired
    bool pending = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<long long> sig;   // what the captured graph was built for
    int persist_blocks = 0;       // workgroups of the persistent launch (all resident)
};

constexpr int kDefaultPassFrames = 8;
constexpr int kMaxWalkChunk = 64;

static LaunchShape default_shape(int cus)
{
    return {cus, cus * 16, cus * 16, 1, 4, 0, 0, cus};
}

struct slim_map {
    slim_map_config cfg;
    int nsem = 0;
    int maxsteps = 0;
    int cus = 256;
    LaunchShape shape = default_shape(256);
    int pass_frames = kDefaultPassFrames;  // frames slim_integrate_sequence integrates in one pass
    BatchCtx *batch = nullptr;
    MapDev md = {};
    size_t hcap = 0;
    size_t pair_cap = 0;
    // second staging buffer and walk stream of slim_integrate_sequence: the
    // walk of frame t + 1 runs beside the rest of frame t
    MapDev md1 = {};
    bool have1 = false;
    size_t pair_cap1 = 0;
    hipStream_t wstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_free[2] = {nullptr, nullptr}, ev_walk[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    // extraction scratch
    unsigned long long *ext_keys = nullptr;
    int32_t *ext_slots = nullptr;
    uint32_t *ext_offsets = nullptr;
    size_t ext_cap = 0;
    // kernel timing
    bool prof = false;
    std::vector<hipEvent_t> ev;  // kProfRing * 2 * kNumProfiled
    int prof_head = 0, prof_count = 0;
    int prof_frames[kProfRing] = {};  // frames of each launch set in the ring
    double prof_ms[kNumProfiled] = {};
    long long prof_n[kNumProfiled] = {};
    // per launch set, until slim_profile_sets reads them
    struct ProfSet {
        int frames;
        double ms[kNumProfiled];
        double span;
    };
    std::vector<ProfSet> prof_sets;
    hipError_t noalloc_err = hipSuccess;  // outcome of the scratch address setup at create
    // loss adjoints (allocated by the first slim_map_loss)
    float *adj = nullptr;
    int32_t *adj_cnt = nullptr;
    float *part = nullptr;
    int32_t *part_cnt = nullptr;
    size_t part_cap = 0;
    std::vector<void *> allocs;
};

namespace {

template <class T>
slim_status dalloc(slim_map *m, T **p, size_t count)
{
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess)
        return fail(SLIM_ERR_DEVICE, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    m->allocs.push_back(q);
    *p = (T *)q;
    return SLIM_OK;
}

void free_batch(slim_map *m)
{
    BatchCtx *b = m->batch;
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->copied) (void)hipEventDestroy(b->copied);
    if (b->dev) (void)hipFree(b->dev);
    if (b->staging) (void)hipHostFree(b->staging);
    delete b;
    m->batch = nullptr;
}

void free_all(slim_map *m)
{
    free_batch(m);
    if (m->wstream) (void)hipStreamDestroy(m->wstream);
    m->wstream = nullptr;
    for (hipEvent_t *e : {&m->ev_in, &m->ev_free[0], &m->ev_free[1], &m->ev_walk[0], &m->ev_walk[1]}) {
        if (*e) (void)hipEventDestroy(*e);
        *e = nullptr;
    }
    for (void *p : m->allocs) (void)hipFree(p);
    m->allocs.clear();
    for (hipEvent_t e : m->ev) (void)hipEventDestroy(e);
    m->ev.clear();
}

slim_status validate_config(const slim_map_config *c)
{
    if (!c) return fail(SLIM_ERR_INVALID, "config is NULL");
    if (!(c->voxel_size > 0.0f) || !std::isfinite(c->voxel_size))
        return fail(SLIM_ERR_INVALID, "voxel_size must be finite and > 0");
    if (!(c->sdf_trunc >= c->voxel_size) || !std::isfinite(c->sdf_trunc))
        return fail(SLIM_ERR_INVALID, "sdf_trunc must be finite and >= voxel_size");
    if (c->sdf_trunc > 6.0f * c->voxel_size)
        return fail(SLIM_ERR_UNSUPPORTED, "sdf_trunc above 6 voxel sizes is not supported");
    if (!(c->min_range >= 0.0f) || !(c->max_range > c->min_range) || !std::isfinite(c->max_range))
        return fail(SLIM_ERR_INVALID, "need 0 <= min_range < max_range < inf");
    if (c->sem_mode == SLIM_SEM_CLOSED || c->sem_mode == SLIM_SEM_CLOSED_LAST) {
        if (c->num_classes < 1 || c->num_classes > 256) return fail(SLIM_ERR_INVALID, "num_classes must be 1..256");
    } else if (c->sem_mode == SLIM_SEM_OPEN || c->sem_mode == SLIM_SEM_OPEN_LAST) {
        if (c->embed_dim < 1 || c->embed_dim > 1024) return fail(SLIM_ERR_INVALID, "embed_dim must be 1..1024");
    } else if (c->sem_mode != SLIM_SEM_NONE) {
        return fail(SLIM_ERR_INVALID, "unknown sem_mode %d", c->sem_mode);
    }
    if (c->max_leaves < 1 || c->max_leaves > (int64_t(1) << 26))
        return fail(SLIM_ERR_INVALID, "max_leaves must be 1..2^26");
    if (c->max_voxels < 1 || c->max_voxels > int64_t(0x7FFFFFFF))
        return fail(SLIM_ERR_INVALID, "max_voxels must be 1..2^31-1");
    if (c->device < 0) return fail(SLIM_ERR_INVALID, "device must be >= 0");
    return SLIM_OK;
}

int max_steps(float vs, float tau)
{
    // the band is at most 2 tau long; 3 * ceil(2 tau / vs) + 4 cells bound its walk
    return 3 * (int)std::ceil((2.0 * (double)tau) / (double)vs) + 4;
}

slim_status ensure_pairs(slim_map *m, size_t need, hipStream_t s, int buf = 0)
{
    size_t &pcap = buf ? m->pair_cap1 : m->pair_cap;
    if (need <= pcap) return SLIM_OK;
    if (need > 0xFFFFFFF0ull) return fail(SLIM_ERR_INVALID, "frame needs more than 2^32 pair slots");
    HIP_OK(hipStreamSynchronize(s));
    if (m->wstream) HIP_OK(hipStreamSynchronize(m->wstream));
    size_t cap = std::max<size_t>(need, pcap + pcap / 2);
    cap = std::min<size_t>(cap, 0xFFFFFFF0ull);
    MapDev &md = buf ? m->md1 : m->md;
    void *ptrs[10] = {md.pairs,   md.pair_key, md.pair_tsdf, md.srt_kv,  md.srt_lab,
                      md.tmp_key, md.tmp_tsdf, md.work,      md.vox_list, md.items_big};
    for (void *p : ptrs) {
        if (!p) continue;
        (void)hipFree(p);
        m->allocs.erase(std::remove(m->allocs.begin(), m->allocs.end(), p), m->allocs.end());
    }
    md.pairs = nullptr;
    md.pair_key = md.tmp_key = nullptr;
    md.pair_tsdf = md.tmp_tsdf = nullptr;
    md.srt_kv = nullptr;
    md.srt_lab = nullptr;
    md.work = nullptr;
    md.vox_list = nullptr;
    md.items_big = nullptr;
    // a large leaf has more than kLeafLdsPairs pairs and at most 8 slab items
    const size_t wcap = cap / (kLeafLdsPairs / kLeafPages) + kLeafPages;
    slim_status r;
    if ((r = dalloc(m, &md.pairs, cap)) ||
        (r = dalloc(m, &md.pair_key, cap)) || (r = dalloc(m, &md.pair_tsdf, cap)) ||
        (r = dalloc(m, &md.srt_kv, cap)) ||
        (r = dalloc(m, &md.srt_lab, cap)) || (r = dalloc(m, &md.tmp_key, cap)) ||
        (r = dalloc(m, &md.tmp_tsdf, cap)) ||
        (r = dalloc(m, &md.work, wcap)) || (r = dalloc(m, &md.vox_list, cap)) ||
        (r = dalloc(m, &md.items_big, wcap))) {
        pcap = 0;
        md.pair_cap = 0;
        md.work_cap = 0;
        return r;
    }
    pcap = cap;
    md.pair_cap = (uint32_t)cap;
    md.work_cap = (uint32_t)wcap;
    return SLIM_OK;
}

// Folds finished timing events into the per-kernel totals.  With wait, waits
// for all of them.
slim_status drain_profile(slim_map *m, bool wait)
{
    while (m->prof_count > 0) {
        const int slot = (m->prof_head - m->prof_count + kProfRing) % kProfRing;
        hipEvent_t *e = &m->ev[(size_t)slot * 2 * kNumProfiled];
        if (!wait && hipEventQuery(e[2 * kNumProfiled - 1]) != hipSuccess) break;
        HIP_OK(hipEventSynchronize(e[2 * kNumProfiled - 1]));
        slim_map::ProfSet set;
        set.frames = m->prof_frames[slot];
        for (int k = 0; k < kNumProfiled; ++k) {
            float ms = 0.0f;
            HIP_OK(hipEventElapsedTime(&ms, e[2 * k], e[2 * k + 1]));
            m->prof_ms[k] += ms;
            m->prof_n[k] += 1;
            set.ms[k] = ms;
        }
        float span = 0.0f;
        HIP_OK(hipEventElapsedTime(&span, e[0], e[2 * kNumProfiled - 1]));
        set.span = span;
        if (m->prof_sets.size() < kMaxProfSets) m->prof_sets.push_back(set);
        m->prof_count--;
    }
    return SLIM_OK;
}

}  // namespace

extern "C" {

const char *slim_last_error(void) { return g_err; }

slim_status slim_map_create(const slim_map_config *config, slim_map **out)
{
    g_err[0] = 0;
    if (!out) return fail(SLIM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    slim_status r = validate_config(config);
    if (r) return r;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(SLIM_ERR_DEVICE, "no HIP device");
    if (config->device >= ndev) return fail(SLIM_ERR_INVALID, "device %d does not exist", config->device);
    DeviceGuard g(config->device);

    slim_map *m = new slim_map();
    m->cfg = *config;
    m->nsem = config->sem_mode == SLIM_SEM_CLOSED        ? config->num_classes
              : config->sem_mode == SLIM_SEM_OPEN        ? 2 * config->embed_dim
              : config->sem_mode == SLIM_SEM_CLOSED_LAST ? 1
              : config->sem_mode == SLIM_SEM_OPEN_LAST   ? config->embed_dim
                                                         : 0;
    m->maxsteps = max_steps(config->voxel_size, config->sdf_trunc);
    if (m->maxsteps > 64) {  // the walk kernel records a ray's cells in 64-bit masks
        delete m;
        return fail(SLIM_ERR_UNSUPPORTED, "sdf_trunc / voxel_size too large");
    }
    size_t cap = 1024;
    while (cap < 2 * (size_t)config->max_leaves) cap <<= 1;
    m->hcap = cap;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, config->device) == hipSuccess && prop.multiProcessorCount > 0)
        m->cus = prop.multiProcessorCount;
    m->shape = default_shape(m->cus);

    MapDev &md = m->md;
    md.hmask = (uint32_t)(cap - 1);
    md.max_leaves = config->max_leaves;
    md.max_pages = (config->max_voxels + kPageVoxels - 1) / kPageVoxels;
    md.rec_stride = record_stride(m->nsem);
    md.leaf_blocks = m->cus * 16;
    md.wave_pairs = 0;
    md.slab_pairs = 0;
    const size_t L = (size_t)config->max_leaves, NP = (size_t)md.max_pages;
    if ((r = dalloc(m, &md.htab, cap)) || (r = dalloc(m, &md.skeys, cap)) ||
        (r = dalloc(m, &md.touched, cap)) || (r = dalloc(m, &md.touched_key, cap)) ||
        (r = dalloc(m, &md.pos_count, cap)) ||
        (r = dalloc(m, &md.pos_slab, cap)) || (r = dalloc(m, &md.pos_plan, cap)) ||
        (r = dalloc(m, &md.pos_pages, 2 * cap)) || (r = dalloc(m, &md.items, cap)) ||
        (r = dalloc(m, &md.items_small, cap)) || (r = dalloc(m, &md.leaf_key, L)) ||
        (r = dalloc(m, &md.leaf_page, L * kLeafPages)) || (r = dalloc(m, &md.leaf_occ, L * kMaskWords)) ||
        (r = dalloc(m, &md.vox, NP * kPageVoxels * (size_t)md.rec_stride)) ||
        (r = dalloc(m, &md.blk_stats, (size_t)m->cus * kMaxLeafBlocksPerCu)) || (r = dalloc(m, &md.st, 1)) ||
        (r = dalloc(m, &md.fs, 1))) {
        free_all(m);
        delete m;
        return r;
    }
    if (launch_reset(md, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        free_all(m);
        delete m;
        return fail(SLIM_ERR_DEVICE, "map initialisation failed");
    }
    // the device address of the allocation-free extract's scratch on this GPU
    // (a failure here is reported by slim_extract_noalloc, not by create)
    m->noalloc_err = noalloc_scratch_setup(config->device);
    *out = m;
    return SLIM_OK;
}

slim_status slim_map_destroy(slim_map *m)
{
    g_err[0] = 0;
    if (!m) return SLIM_OK;
    {
        DeviceGuard g(m->cfg.device);
        (void)hipDeviceSynchronize();
        free_all(m);
    }
    delete m;
    return SLIM_OK;
}

slim_status slim_map_reset(slim_map *m, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    DeviceGuard g(m->cfg.device);
    HIP_OK(launch_reset(m->md, (hipStream_t)stream));
    if (m->have1) {
        // the second buffer's last walk and commit are done before it is cleared
        if (m->used[1]) HIP_OK(hipStreamWaitEvent((hipStream_t)stream, m->ev_free[1], 0));
        HIP_OK(launch_reset_staging(m->md1, (hipStream_t)stream));
        HIP_OK(hipEventRecord(m->ev_free[1], (hipStream_t)stream));
        m->used[1] = true;
    }
    return SLIM_OK;
}

}  // extern "C"

namespace {

// Validates a frame and canonicalises its pose (FP64 -> anchor voxel + FP32).
slim_status make_frame(slim_map *m, const float *points, const float *ranges, const float *dirs, int64_t n,
                       const double *pose, const void *sem, int32_t kind, FrameParams *fp)
{
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (n < 0 || n >= kMaxPoints) return fail(SLIM_ERR_INVALID, "n must be in [0, 2^23)");
    if (n > 0 && !points && !(ranges && dirs)) return fail(SLIM_ERR_INVALID, "points are NULL");
    if (((uintptr_t)points & 3u) != 0 || ((uintptr_t)ranges & 3u) != 0 || ((uintptr_t)dirs & 3u) != 0)
        return fail(SLIM_ERR_INVALID, "points must be 4-byte aligned");
    if (!pose) return fail(SLIM_ERR_INVALID, "pose is NULL");
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(pose[i])) return fail(SLIM_ERR_INVALID, "pose has a non-finite entry");
    const slim_map_config &c = m->cfg;
    bool kind_ok = false;
    if (c.sem_mode == SLIM_SEM_NONE) kind_ok = kind == SLIM_IN_NONE;
    const bool closed = c.sem_mode == SLIM_SEM_CLOSED || c.sem_mode == SLIM_SEM_CLOSED_LAST;
    const bool open = c.sem_mode == SLIM_SEM_OPEN || c.sem_mode == SLIM_SEM_OPEN_LAST;
    const bool last = c.sem_mode == SLIM_SEM_CLOSED_LAST || c.sem_mode == SLIM_SEM_OPEN_LAST;
    if (closed) kind_ok = kind == SLIM_IN_LABEL_I32 || kind == SLIM_IN_PROB_F32 || kind == SLIM_IN_LOGIT_F32;
    if (open) kind_ok = kind == SLIM_IN_EMB_BF16 || kind == SLIM_IN_EMB_F32;
    if (!kind_ok) return fail(SLIM_ERR_INVALID, "semantic input kind %d does not match the map's mode", kind);
    if (kind == SLIM_IN_LOGIT_F32 && !last && c.num_classes > 64)
        return fail(SLIM_ERR_UNSUPPORTED, "logit input supports at most 64 classes");
    if (kind != SLIM_IN_NONE && n > 0 && !sem) return fail(SLIM_ERR_INVALID, "semantic input is NULL");
    if (((uintptr_t)sem & (kind == SLIM_IN_EMB_BF16 ? 1u : 3u)) != 0)
        return fail(SLIM_ERR_INVALID, "semantic input is misaligned");

    // anchor voxel of the sensor origin; an origin 2^20 or more voxels out is
    // anchored at +2^20, where every point whose walk leaves |k| < 2^20 is
    // rejected on its own
    const double vsd = (double)c.voxel_size;
    for (int r = 0; r < 3; ++r) {
        const double ta = pose[4 * r + 3];
        double q = std::floor(ta / vsd);
        if (!(std::fabs(q) < (double)kKeyLimit)) q = (double)kKeyLimit;
        fp->a[r] = (int)q;
        fp->t[r] = (float)(ta - (double)fp->a[r] * vsd);
        for (int k = 0; k < 3; ++k) fp->R[3 * r + k] = (float)pose[4 * r + k];
    }
    fp->vs = c.voxel_size;
    fp->tau = c.sdf_trunc;
    fp->rmin = c.min_range;
    fp->rmax = c.max_range;
    fp->maxsteps = m->maxsteps;
    fp->n = (int)n;
    fp->sem_kind = kind;
    fp->K = closed ? c.num_classes : 0;
    fp->L = open ? c.embed_dim : 0;
    fp->last = last ? 1 : 0;
    fp->nsem = m->nsem;
    fp->pts = points;
    fp->ranges = points ? nullptr : ranges;
    fp->dirs = points ? nullptr : dirs;
    fp->depth = nullptr;
    fp->width = 0;
    fp->fx = fp->fy = fp->cx = fp->cy = 0.0f;
    fp->sem = sem;
    fp->pid_base = 0;
    fp->nsub = 0;
    fp->pass_first = 0;
    for (int f = 0; f <= kPassFrames; ++f) fp->sub_start[f] = 0;
    for (int f = 0; f < kPassFrames; ++f) fp->sub_sem[f] = nullptr;
    return SLIM_OK;
}

// One frame, or with pw the frames of a multi-frame pass (fp then describes the
// pass: n is its total of points), with kernel timing events while enabled.
slim_status integrate_frame(slim_map *m, const FrameParams &fp, void *stream, const PassWalk *pw = nullptr)
{
    DeviceGuard g(m->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    slim_status r = ensure_pairs(m, (size_t)std::max<int>(fp.n, 1) * (size_t)m->maxsteps, s);
    if (r) return r;
    hipEvent_t *ev = nullptr;
    if (m->prof) {
        if (m->prof_count == kProfRing) {
            r = drain_profile(m, false);
            if (r) return r;
            if (m->prof_count == kProfRing) {
                // oldest frame still running: wait for it
                const int slot = (m->prof_head - m->prof_count + kProfRing) % kProfRing;
                HIP_OK(hipEventSynchronize(m->ev[(size_t)slot * 2 * kNumProfiled + 2 * kNumProfiled - 1]));
                r = drain_profile(m, false);
                if (r) return r;
            }
        }
        ev = &m->ev[(size_t)m->prof_head * 2 * kNumProfiled];
        m->prof_frames[m->prof_head] = fp.nsub > 1 ? fp.nsub : 1;
        m->prof_head = (m->prof_head + 1) % kProfRing;
        m->prof_count++;
    }
    HIP_OK(launch_integrate(fp, m->md, m->shape, s, ev, pw));
    return SLIM_OK;
}

// The second staging buffer: its own staging table, counts, plans, items and
// frame counters (pair buffers come from ensure_pairs), the map's arrays shared.
slim_status ensure_buffer1(slim_map *m, hipStream_t s)
{
    if (m->have1) return SLIM_OK;
    MapDev md = m->md;
    md.skeys = nullptr;
    md.touched = md.pos_count = md.pos_slab = nullptr;
    md.touched_key = nullptr;
    md.pos_plan = md.pos_pages = nullptr;
    md.items = md.items_small = nullptr;
    md.fs = nullptr;
    md.pairs = nullptr;
    md.pair_key = md.tmp_key = nullptr;
    md.pair_tsdf = md.tmp_tsdf = nullptr;
    md.srt_kv = nullptr;
    md.srt_lab = nullptr;
    md.work = nullptr;
    md.vox_list = nullptr;
    md.items_big = nullptr;
    md.pair_cap = 0;
    md.work_cap = 0;
    const size_t cap = m->hcap;
    slim_status r;
    if ((r = dalloc(m, &md.skeys, cap)) || (r = dalloc(m, &md.touched, cap)) ||
        (r = dalloc(m, &md.touched_key, cap)) || (r = dalloc(m, &md.pos_count, cap)) ||
        (r = dalloc(m, &md.pos_slab, cap)) || (r = dalloc(m, &md.pos_plan, cap)) ||
        (r = dalloc(m, &md.pos_pages, 2 * cap)) || (r = dalloc(m, &md.items, cap)) ||
        (r = dalloc(m, &md.items_small, cap)) || (r = dalloc(m, &md.fs, 1)))
        return r;
    HIP_OK(hipStreamCreateWithFlags(&m->wstream, hipStreamNonBlocking));
    // these events only order work between the map's two streams on the GPU:
    // device-scope release, no system-scope cache writeback at each record
    for (hipEvent_t *e : {&m->ev_in, &m->ev_free[0], &m->ev_free[1], &m->ev_walk[0], &m->ev_walk[1]})
        HIP_OK(hipEventCreateWithFlags(e, hipEventDisableTiming | hipEventReleaseToDevice));
    HIP_OK(launch_reset_staging(md, s));
    m->md1 = md;
    m->pair_cap1 = 0;
    m->used[0] = m->used[1] = false;
    m->have1 = true;
    return SLIM_OK;
}

// Frames [t0, t1) of a sequence, one at a time, with the walk of frame t + 1
// on the walk stream beside the rest of frame t (two staging buffers).
slim_status integrate_overlapped(slim_map *m, const std::vector<FrameParams> &fps, int t0, int t1, hipStream_t s)
{
    if (t1 - t0 == 1) return integrate_frame(m, fps[t0], s);
    slim_status r = ensure_buffer1(m, s);
    if (r) return r;
    int64_t nmax = 1;
    for (int t = t0; t < t1; ++t) nmax = std::max<int64_t>(nmax, fps[t].n);
    const size_t need = (size_t)nmax * (size_t)m->maxsteps;
    if ((r = ensure_pairs(m, need, s, 0)) || (r = ensure_pairs(m, need, s, 1))) return r;
    // every frame's inputs, and all earlier work on the stream, come first
    HIP_OK(hipEventRecord(m->ev_in, s));
    HIP_OK(hipStreamWaitEvent(m->wstream, m->ev_in, 0));
    for (int t = t0; t < t1; ++t) {
        const int b = t & 1;
        const MapDev &md = b ? m->md1 : m->md;
        // the walk of frame t (on the walk stream) needs only its buffer back
        // from frame t - 2; the rest of the frame follows frame t - 1 in order
        if (m->used[b]) HIP_OK(hipStreamWaitEvent(m->wstream, m->ev_free[b], 0));
        HIP_OK(launch_walk(fps[t], md, m->wstream));
        HIP_OK(hipEventRecord(m->ev_walk[b], m->wstream));
        HIP_OK(hipStreamWaitEvent(s, m->ev_walk[b], 0));
        HIP_OK(launch_after_walk(fps[t], md, m->shape, s));
        HIP_OK(hipEventRecord(m->ev_free[b], s));
        m->used[b] = true;
    }
    return SLIM_OK;
}

// Frames a multi-frame pass can take: geometry, or int32 labels with at most
// 32 classes, Bayesian mode.

// The pass of frames [t0, t1): its walk (each frame's rays, point indices
// offset per frame so that every observation key stays distinct and
// frame-ordered) and the frame parameters of the rest of its kernels, which
// run once for the union of the leaves the frames touch.
void make_pass(const std::vector<FrameParams> &fps, int t0, int t1, FrameParams *base, PassWalk *pw)
{
    memset(pw, 0, sizeof(*pw));
    *base = fps[t0];
    uint32_t off = 0;
    int nb = 0;
    for (int f = 0; f < t1 - t0; ++f) {
        FrameParams fp = fps[t0 + f];
        fp.pid_base = off;
        pw->fp[f] = fp;
        pw->blk_start[f] = nb;
        nb += (fp.n + kWalkThreads - 1) / kWalkThreads;
        base->sub_start[f] = off;
        base->sub_sem[f] = fp.sem;
        off += (uint32_t)fp.n;
    }
    pw->blk_start[t1 - t0] = nb;
    pw->nframes = t1 - t0;
    base->sub_start[t1 - t0] = off;
    base->nsub = t1 - t0;
    base->pass_first = t0;
    base->n = (int)off;
}

// A sequence in passes of up to m->pass_frames consecutive frames (the last
// frame alone, so that the per-frame statistics are its own).  Without kernel
// timing, passes alternate between the two staging buffers and the walk of
// pass p + 1 runs on the walk stream beside the rest of pass p.  A pass the
// map cannot take (capacity, staging) is not applied, nor is anything after
// it; after the queue drains, those frames are integrated again one at a
// time, which reproduces exactly what per-frame calls do.
slim_status integrate_passes(slim_map *m, const std::vector<FrameParams> &fps, hipStream_t s)
{
    const int count = (int)fps.size();
    std::vector<std::pair<int, int>> units;
    int64_t most = 1;
    for (int t = 0; t < count;) {
        int t1 = t + 1;
        int64_t tot = fps[t].n;
        while (t < count - 1 && t1 < count - 1 && t1 - t < std::min(m->pass_frames, kAccFrames) &&
               fps[t1].sem_kind == fps[t].sem_kind &&
               tot + fps[t1].n < kMaxPoints) {
            tot += fps[t1].n;
            ++t1;
        }
        units.emplace_back(t, t1);
        most = std::max<int64_t>(most, tot);
        t = t1;
    }
    slim_status r = SLIM_OK;
    FrameParams base;
    PassWalk pw;
    if (m->prof) {
        for (const auto &u : units) {
            if (u.second - u.first == 1) {
                r = integrate_frame(m, fps[u.first], s);
            } else {
                make_pass(fps, u.first, u.second, &base, &pw);
                r = integrate_frame(m, base, s, &pw);
            }
            if (r) break;
        }
    } else {
        const size_t need = (size_t)most * (size_t)m->maxsteps;
        if (!(r = ensure_buffer1(m, s)) && !(r = ensure_pairs(m, need, s, 0)) && !(r = ensure_pairs(m, need, s, 1))) {
            HIP_OK(hipEventRecord(m->ev_in, s));
            HIP_OK(hipStreamWaitEvent(m->wstream, m->ev_in, 0));
            for (size_t i = 0; i < units.size(); ++i) {
                const int b = (int)(i & 1);
                const MapDev &md = b ? m->md1 : m->md;
                const bool pass = units[i].second - units[i].first > 1;
                if (pass) make_pass(fps, units[i].first, units[i].second, &base, &pw);
                const FrameParams &fp = pass ? base : fps[units[i].first];
                if (m->used[b]) HIP_OK(hipStreamWaitEvent(m->wstream, m->ev_free[b], 0));
                HIP_OK(launch_walk(fp, md, m->wstream, pass ? &pw : nullptr));
                HIP_OK(hipEventRecord(m->ev_walk[b], m->wstream));
                HIP_OK(hipStreamWaitEvent(s, m->ev_walk[b], 0));
                HIP_OK(launch_after_walk(fp, md, m->shape, s));
                HIP_OK(hipEventRecord(m->ev_free[b], s));
                m->used[b] = true;
            }
        }
    }
    // whatever was queued has run once the stream drains; a pass that was not
    // applied leaves its first frame in pass_failed
    int failed = 0;
    HIP_OK(hipMemcpyAsync(&failed, &m->md.st->pass_failed, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (failed == 0) return r;
    HIP_OK(hipMemsetAsync(&m->md.st->pass_failed, 0, sizeof(int), s));
    if (r) return r;
    return integrate_overlapped(m, fps, failed - 1, count, s);
}

}  // namespace

extern "C" {

slim_status slim_integrate_sequence(slim_map *m, const slim_frame *frames, int32_t count, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (count < 0 || (count > 0 && !frames)) return fail(SLIM_ERR_INVALID, "need count >= 0 and frames");
    if (count == 0) return SLIM_OK;
    DeviceGuard g(m->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    std::vector<FrameParams> fps(count);
    for (int i = 0; i < count; ++i) {
        const slim_frame &f = frames[i];
        if (f.points && (f.ranges || f.dirs)) return fail(SLIM_ERR_INVALID, "frame %d has points and rays", i);
        if (f.n > 0 && !f.points && !(f.ranges && f.dirs)) return fail(SLIM_ERR_INVALID, "frame %d has no points", i);
        slim_status r = make_frame(m, f.points, f.ranges, f.dirs, f.n, f.pose, f.sem, f.sem_kind, &fps[i]);
        if (r) return r;
    }
    if (count == 1) return integrate_frame(m, fps[0], stream);
    if (m->pass_frames > 1 && count > 2) {
        bool all = true;
        for (int i = 0; i < count && all; ++i) all = accum_path(fps[i]);
        if (all) return integrate_passes(m, fps, s);
    }
    return integrate_overlapped(m, fps, 0, count, s);
}

slim_status slim_integrate(slim_map *m, const float *points, int64_t n, const double *pose, const void *sem,
                           int32_t kind, void *stream)
{
    g_err[0] = 0;
    if (m && n > 0 && !points) return fail(SLIM_ERR_INVALID, "points is NULL");
    FrameParams fp;
    slim_status r = make_frame(m, points, nullptr, nullptr, n, pose, sem, kind, &fp);
    return r ? r : integrate_frame(m, fp, stream);
}

slim_status slim_integrate_rays(slim_map *m, const float *ranges, const float *dirs, int64_t n, const double *pose,
                                const void *sem, int32_t kind, void *stream)
{
    g_err[0] = 0;
    if (m && n > 0 && (!ranges || !dirs)) return fail(SLIM_ERR_INVALID, "ranges or directions are NULL");
    FrameParams fp;
    slim_status r = make_frame(m, nullptr, ranges, dirs, n, pose, sem, kind, &fp);
    return r ? r : integrate_frame(m, fp, stream);
}

slim_status slim_integrate_depth(slim_map *m, const float *depth, int32_t width, int32_t height,
                                 const float *intrinsics, const double *pose, const void *sem, int32_t kind,
                                 void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (width < 0 || height < 0) return fail(SLIM_ERR_INVALID, "width and height must be >= 0");
    const int64_t n = (int64_t)width * height;
    if (n >= kMaxPoints) return fail(SLIM_ERR_INVALID, "width * height must be below 2^23");
    if (n > 0 && !depth) return fail(SLIM_ERR_INVALID, "depth is NULL");
    if (((uintptr_t)depth & 3u) != 0) return fail(SLIM_ERR_INVALID, "depth must be 4-byte aligned");
    if (!intrinsics) return fail(SLIM_ERR_INVALID, "intrinsics are NULL");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(intrinsics[i])) return fail(SLIM_ERR_INVALID, "intrinsics must be finite");
    if (!(intrinsics[0] != 0.0f && intrinsics[1] != 0.0f)) return fail(SLIM_ERR_INVALID, "fx and fy must be nonzero");
    if (kind != SLIM_IN_NONE && n > 0 && !sem) return fail(SLIM_ERR_INVALID, "semantic input is NULL");
    FrameParams fp;
    slim_status r = make_frame(m, nullptr, nullptr, nullptr, 0, pose, sem, kind, &fp);
    if (r) return r;
    fp.n = (int)n;
    fp.depth = depth;
    fp.width = width;
    fp.fx = intrinsics[0];
    fp.fy = intrinsics[1];
    fp.cx = intrinsics[2];
    fp.cy = intrinsics[3];
    return integrate_frame(m, fp, stream);
}

slim_status slim_map_stats(slim_map *m, slim_stats *out, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (!out) return fail(SLIM_ERR_INVALID, "out is NULL");
    DeviceGuard g(m->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    DevState st;
    HIP_OK(hipMemcpyAsync(&st, m->md.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    out->leaves = (int64_t)st.leaves_used;
    out->voxels = (int64_t)st.voxels_used;
    out->points_last = st.last_points;
    out->rejected_last = st.last_rejected;
    out->pairs_last = st.last_pairs;
    out->touched_leaves_last = st.last_touched;
    out->new_leaves_last = st.last_new_leaves;
    out->voxels_old_last = st.last_u_old;
    out->voxels_new_last = st.last_u_new;
    out->status_last = st.last_status;
    out->reserved = 0;
    if (st.status != SLIM_OK) {
        const int zero = 0;
        HIP_OK(hipMemcpyAsync(&m->md.st->status, &zero, sizeof(int), hipMemcpyHostToDevice, s));
        HIP_OK(hipStreamSynchronize(s));
        return fail(st.status, "a queued frame failed on the GPU (%s)",
                    st.status == SLIM_ERR_CAPACITY ? "leaf or voxel capacity exceeded; frame not applied"
                                                   : "device error");
    }
    return SLIM_OK;
}

slim_status slim_extract(slim_map *m, int64_t capacity, int32_t *keys, float *d, float *w, float *sem,
                         int64_t *count, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (!count) return fail(SLIM_ERR_INVALID, "count is NULL");
    slim_stats st;
    slim_status r = slim_map_stats(m, &st, stream);
    if (r) return r;
    *count = st.voxels;
    if (capacity == 0) return SLIM_OK;
    if (capacity < st.voxels) return fail(SLIM_ERR_INVALID, "capacity %lld < voxel count %lld",
                                          (long long)capacity, (long long)st.voxels);
    if (st.voxels > 0 && (!keys || !d || !w)) return fail(SLIM_ERR_INVALID, "output pointer is NULL");
    DeviceGuard g(m->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    if ((size_t)st.leaves > m->ext_cap) {
        HIP_OK(hipStreamSynchronize(s));
        for (void *p : {(void *)m->ext_keys, (void *)m->ext_slots, (void *)m->ext_offsets}) {
            if (!p) continue;
            (void)hipFree(p);
            m->allocs.erase(std::remove(m->allocs.begin(), m->allocs.end(), p), m->allocs.end());
        }
        m->ext_keys = nullptr;
        m->ext_slots = nullptr;
        m->ext_offsets = nullptr;
        m->ext_cap = 0;
        const size_t cap = (size_t)st.leaves;
        if ((r = dalloc(m, &m->ext_keys, cap)) || (r = dalloc(m, &m->ext_slots, cap)) ||
            (r = dalloc(m, &m->ext_offsets, cap)))
            return r;
        m->ext_cap = cap;
    }
    HIP_OK(launch_extract(m->md, m->nsem, st.leaves, m->ext_keys, m->ext_slots, m->ext_offsets, keys, d, w,
                          m->nsem ? sem : nullptr, s));
    HIP_OK(hipStreamSynchronize(s));
    return SLIM_OK;
}

slim_status slim_extract_noalloc(slim_map *m, int64_t capacity, int32_t *keys, float *d, float *w, float *sem,
                                 int64_t *count, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (!count) return fail(SLIM_ERR_INVALID, "count is NULL");
    slim_stats st;
    slim_status r = slim_map_stats(m, &st, stream);
    if (r) return r;
    *count = st.voxels;
    if (capacity == 0) return SLIM_OK;
    if (capacity < st.voxels) return fail(SLIM_ERR_INVALID, "capacity %lld < voxel count %lld",
                                          (long long)capacity, (long long)st.voxels);
    if (st.voxels > 0 && (!keys || !d || !w)) return fail(SLIM_ERR_INVALID, "output pointer is NULL");
    if (st.leaves > kNoAllocMaxLeaves)
        return fail(SLIM_ERR_CAPACITY, "the map has %lld leaves; slim_extract_noalloc handles at most %lld",
                    (long long)st.leaves, kNoAllocMaxLeaves);
    if (m->noalloc_err != hipSuccess)
        return fail(SLIM_ERR_DEVICE, "scratch address of device %d unavailable: %s", m->cfg.device,
                    hipGetErrorString(m->noalloc_err));
    void *ptr = noalloc_scratch(m->cfg.device);
    if (!ptr) return fail(SLIM_ERR_DEVICE, "scratch address of device %d unavailable", m->cfg.device);
    DeviceGuard g(m->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    // keys, slots and offsets of the leaves, each array sized for the maximum;
    // every entry the kernels read is written first by this call
    unsigned long long *tk = (unsigned long long *)ptr;
    int32_t *ts = (int32_t *)(tk + kNoAllocMaxLeaves);
    uint32_t *to = (uint32_t *)(ts + kNoAllocMaxLeaves);
    HIP_OK(launch_extract(m->md, m->nsem, st.leaves, tk, ts, to, keys, d, w, m->nsem ? sem : nullptr, s));
    HIP_OK(hipStreamSynchronize(s));
    return SLIM_OK;
}

slim_status slim_query(slim_map *m, const float *xyz, int64_t mq, float *d, float *w, float *sem, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (mq < 0) return fail(SLIM_ERR_INVALID, "m must be >= 0");
    if (mq > 0 && (!xyz || !d || !w)) return fail(SLIM_ERR_INVALID, "a pointer is NULL");
    DeviceGuard g(m->cfg.device);
    HIP_OK(launch_query(m->md, m->nsem, m->cfg.voxel_size, xyz, mq, d, w, m->nsem ? sem : nullptr,
                        (hipStream_t)stream));
    return SLIM_OK;
}

slim_status slim_predict(slim_map *m, const float *xyz, int64_t mq, const slim_predict_params *params, float *prob,
                         int32_t *label, float *var, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (!params) return fail(SLIM_ERR_INVALID, "params is NULL");
    if (mq < 0) return fail(SLIM_ERR_INVALID, "m must be >= 0");
    if (mq > 0 && !xyz) return fail(SLIM_ERR_INVALID, "xyz is NULL");
    const int mode = m->cfg.sem_mode;
    if (mode == SLIM_SEM_NONE) return fail(SLIM_ERR_UNSUPPORTED, "a geometry-only map has no semantics");
    const bool open = mode == SLIM_SEM_OPEN || mode == SLIM_SEM_OPEN_LAST;
    if (!std::isfinite(params->threshold)) return fail(SLIM_ERR_INVALID, "threshold must be finite");
    if (mode == SLIM_SEM_CLOSED && !(params->alpha0 > 0.0f && std::isfinite(params->alpha0)))
        return fail(SLIM_ERR_INVALID, "alpha0 must be finite and > 0");
    if (open) {
        if (!(params->temperature > 0.0f && std::isfinite(params->temperature)))
            return fail(SLIM_ERR_INVALID, "temperature must be finite and > 0");
        if (params->num_prototypes < 1 || params->num_prototypes > 1024)
            return fail(SLIM_ERR_INVALID, "num_prototypes must be 1..1024");
        if (!params->prototypes_dev) return fail(SLIM_ERR_INVALID, "prototypes are NULL");
    }
    if (var && mode != SLIM_SEM_OPEN) return fail(SLIM_ERR_UNSUPPORTED, "variances exist for open-set maps only");
    DeviceGuard g(m->cfg.device);
    PredictParams pp = {};
    pp.vs = m->cfg.voxel_size;
    pp.alpha0 = params->alpha0;
    pp.inv_temp = open ? 1.0f / params->temperature : 0.0f;
    pp.threshold = params->threshold;
    pp.mode = mode;
    pp.K = open ? 0 : m->cfg.num_classes;
    pp.L = open ? m->cfg.embed_dim : 0;
    pp.P = open ? params->num_prototypes : 0;
    pp.protos = open ? params->prototypes_dev : nullptr;
    HIP_OK(launch_predict(m->md, pp, xyz, mq, prob, label, var, (hipStream_t)stream));
    return SLIM_OK;
}

slim_status slim_render(slim_map *m, const double *pose, const float *intrinsics, int32_t width, int32_t height,
                        float near_dist, float far_dist, float *depth, int32_t *key, int32_t *label, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (!pose || !intrinsics) return fail(SLIM_ERR_INVALID, "pose or intrinsics are NULL");
    if (width < 0 || height < 0 || (int64_t)width * height > (int64_t(1) << 28))
        return fail(SLIM_ERR_INVALID, "width and height must be >= 0 with at most 2^28 pixels");
    if ((int64_t)width * height > 0 && !depth) return fail(SLIM_ERR_INVALID, "depth is NULL");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(intrinsics[i])) return fail(SLIM_ERR_INVALID, "intrinsics must be finite");
    if (!(intrinsics[0] != 0.0f && intrinsics[1] != 0.0f)) return fail(SLIM_ERR_INVALID, "fx and fy must be nonzero");
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(pose[i])) return fail(SLIM_ERR_INVALID, "pose has a non-finite entry");
    const float vs = m->cfg.voxel_size;
    if (!(near_dist >= 0.0f) || !(far_dist > near_dist) || !std::isfinite(far_dist))
        return fail(SLIM_ERR_INVALID, "need 0 <= near < far < inf");
    if (((double)far_dist - (double)near_dist) / (double)vs >= (double)(1 << 19))
        return fail(SLIM_ERR_INVALID, "far - near must be below 2^19 voxel sizes");
    RenderParams rp = {};
    const double vsd = (double)vs;
    for (int r = 0; r < 3; ++r) {
        const double ta = pose[4 * r + 3];
        const double q = std::floor(ta / vsd);
        if (!(std::fabs(q) < (double)(1 << 19)))
            return fail(SLIM_ERR_INVALID, "pose translation beyond 2^19 voxel sizes");
        rp.a[r] = (int)q;
        rp.t[r] = (float)(ta - (double)rp.a[r] * vsd);
        for (int k = 0; k < 3; ++k) rp.R[3 * r + k] = (float)pose[4 * r + k];
    }
    rp.vs = vs;
    rp.fx = intrinsics[0];
    rp.fy = intrinsics[1];
    rp.cx = intrinsics[2];
    rp.cy = intrinsics[3];
    rp.t0 = near_dist;
    rp.t1 = far_dist;
    rp.maxsteps = 3 * (int)std::ceil(((double)far_dist - (double)near_dist) / vsd) + 4;
    rp.width = width;
    rp.height = height;
    rp.mode = m->cfg.sem_mode;
    rp.K = m->cfg.num_classes;
    DeviceGuard g(m->cfg.device);
    HIP_OK(launch_render(m->md, rp, depth, key, label, (hipStream_t)stream));
    return SLIM_OK;
}

slim_status slim_map_loss(slim_map *m, const int32_t *keys, const int32_t *labels, int64_t mv, const float *samples,
                          int64_t ns, float alpha0, float *loss, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (m->cfg.sem_mode != SLIM_SEM_CLOSED) return fail(SLIM_ERR_UNSUPPORTED, "the map loss needs a closed-set map");
    if (mv < 1 || ns < 0) return fail(SLIM_ERR_INVALID, "need m >= 1 and s >= 0");
    if (!keys || !labels || !loss || (ns > 0 && !samples)) return fail(SLIM_ERR_INVALID, "a pointer is NULL");
    if (!(alpha0 >= 0.0f) || !std::isfinite(alpha0)) return fail(SLIM_ERR_INVALID, "alpha0 must be finite and >= 0");
    DeviceGuard g(m->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    MapDev &md = m->md;
    const size_t nrec = (size_t)md.max_pages * kPageVoxels;
    const int astride = (m->cfg.num_classes + 1 + 3) & ~3;
    slim_status r;
    if (!m->adj) {
        HIP_OK(hipStreamSynchronize(s));
        if ((r = dalloc(m, &m->adj, nrec * astride)) || (r = dalloc(m, &m->adj_cnt, nrec))) return r;
    }
    const size_t nparts = (size_t)((ns + kLossThreads - 1) / kLossThreads + (mv + kLossThreads - 1) / kLossThreads);
    if (nparts > m->part_cap) {
        HIP_OK(hipStreamSynchronize(s));
        for (void *p : {(void *)m->part, (void *)m->part_cnt}) {
            if (!p) continue;
            (void)hipFree(p);
            m->allocs.erase(std::remove(m->allocs.begin(), m->allocs.end(), p), m->allocs.end());
        }
        m->part = nullptr;
        m->part_cnt = nullptr;
        m->part_cap = 0;
        if ((r = dalloc(m, &m->part, nparts)) || (r = dalloc(m, &m->part_cnt, nparts))) return r;
        m->part_cap = nparts;
    }
    LossParams lp;
    lp.keys = keys;
    lp.labels = labels;
    lp.m = mv;
    lp.samples = samples;
    lp.s = ns;
    lp.alpha0 = alpha0;
    lp.loss = loss;
    lp.adj = m->adj;
    lp.adj_cnt = m->adj_cnt;
    lp.adj_stride = astride;
    lp.part = m->part;
    lp.part_cnt = m->part_cnt;
    FrameParams fp = {};
    fp.vs = m->cfg.voxel_size;
    fp.K = m->cfg.num_classes;
    HIP_OK(launch_loss(fp, md, lp, s));
    return SLIM_OK;
}

slim_status slim_backward_rays(slim_map *m, const float *ranges, const float *dirs, int64_t n, const double *pose,
                               const float *logits, const float *grad_scale, float *grad_logits, float *grad_ranges,
                               void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (!m->adj) return fail(SLIM_ERR_INVALID, "no loss has been computed on this map");
    if (m->cfg.num_classes > 32) return fail(SLIM_ERR_UNSUPPORTED, "the backward supports at most 32 classes");
    if (n > 0 && (!ranges || !dirs || !grad_logits || !grad_ranges))
        return fail(SLIM_ERR_INVALID, "a pointer is NULL");
    FrameParams fp;
    slim_status r = make_frame(m, nullptr, ranges, dirs, n, pose, logits, SLIM_IN_LOGIT_F32, &fp);
    if (r) return r;
    DeviceGuard g(m->cfg.device);
    LossParams lp = {};
    lp.adj = m->adj;
    lp.adj_cnt = m->adj_cnt;
    lp.adj_stride = (m->cfg.num_classes + 1 + 3) & ~3;
    HIP_OK(launch_backward(fp, m->md, lp, grad_scale, grad_logits, grad_ranges, (hipStream_t)stream));
    return SLIM_OK;
}

slim_status slim_set_launch_shape(slim_map *m, const slim_launch_shape *shape)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (!shape) {
        m->shape = default_shape(m->cus);
        m->pass_frames = kDefaultPassFrames;
        return SLIM_OK;
    }
    if (shape->plan_blocks < 1 || shape->bucket_blocks < 1 || shape->leaf_blocks_per_cu < 1 ||
        shape->plan_blocks > 65536 || shape->bucket_blocks > 65536 ||
        shape->leaf_blocks_per_cu > kMaxLeafBlocksPerCu || shape->pass_frames < 0 ||
        shape->pass_frames > kPassFrames || shape->batch_mode < 0 || shape->batch_mode > 2 ||
        shape->walk_chunk < 0 || shape->walk_chunk > kMaxWalkChunk ||
        (shape->wave_pairs != 0 && (shape->wave_pairs < 16 || shape->wave_pairs > 256)) ||
        (shape->slab_pairs != 0 && (shape->slab_pairs < 512 || shape->slab_pairs > 2048)))
        return fail(SLIM_ERR_INVALID, "launch shape out of range");
    const LaunchShape d = default_shape(m->cus);
    m->shape = {shape->plan_blocks, shape->bucket_blocks, shape->leaf_blocks_per_cu * m->cus,
                shape->batch_mode == 0 ? d.persistent : (shape->batch_mode == 1 ? 1 : 0),
                shape->walk_chunk > 0 ? shape->walk_chunk : d.walk_chunk, shape->wave_pairs, shape->slab_pairs,
                m->cus};
    m->pass_frames = shape->pass_frames > 0 ? shape->pass_frames : kDefaultPassFrames;
    return SLIM_OK;
}

slim_status slim_integrate_batched(slim_map *const *maps, int32_t nmaps, const slim_frame *frames, int32_t use_graph,
                                   void *stream)
{
    g_err[0] = 0;
    if (!maps || !frames || nmaps < 1 || nmaps > 1024) return fail(SLIM_ERR_INVALID, "need 1..1024 maps and frames");
    for (int i = 0; i < nmaps; ++i) {
        if (!maps[i]) return fail(SLIM_ERR_INVALID, "map %d is NULL", i);
        if (maps[i]->cfg.device != maps[0]->cfg.device) return fail(SLIM_ERR_INVALID, "maps on different devices");
        for (int k = 0; k < i; ++k)
            if (maps[k] == maps[i]) return fail(SLIM_ERR_INVALID, "map %d appears twice", i);
    }
    slim_map *m0 = maps[0];
    DeviceGuard g(m0->cfg.device);
    hipStream_t s = (hipStream_t)stream;
    std::vector<FrameParams> fps(nmaps);
    std::vector<MapDev> mds(nmaps);
    std::vector<int> start(nmaps + 1), kinds(nmaps), subset;
    BatchPlan plan = {};
    plan.nmaps = nmaps;
    start[0] = 0;
    for (int i = 0; i < nmaps; ++i) {
        const slim_frame &f = frames[i];
        if (f.points && (f.ranges || f.dirs)) return fail(SLIM_ERR_INVALID, "frame %d has points and rays", i);
        slim_status r = make_frame(maps[i], f.points, f.ranges, f.dirs, f.n, f.pose, f.sem, f.sem_kind, &fps[i]);
        if (r) return r;
        if (f.n > 0 && !f.points && !(f.ranges && f.dirs)) return fail(SLIM_ERR_INVALID, "frame %d has no points", i);
        r = ensure_pairs(maps[i], (size_t)std::max<int64_t>(f.n, 1) * (size_t)maps[i]->maxsteps, s);
        if (r) return r;
        mds[i] = maps[i]->md;
        mds[i].leaf_blocks = m0->shape.leaf_blocks;
        mds[i].wave_pairs = m0->shape.wave_pairs;
        mds[i].slab_pairs = m0->shape.slab_pairs;
        start[i + 1] = start[i] + (int)std::max<int64_t>(1, (f.n + kWalkThreads - 1) / kWalkThreads);
        kinds[i] = leaf_kernel_kind(fps[i]);
    }
    plan.walk_blocks = start[nmaps];
    // group the maps by leaf-kernel variant
    static_assert(kLeafKinds <= (int)(sizeof(plan.group_kind) / sizeof(int)), "group arrays too small");
    for (int kind = 0; kind < kLeafKinds; ++kind) {
        const int begin = (int)subset.size();
        for (int i = 0; i < nmaps; ++i)
            if (kinds[i] == kind) subset.push_back(i);
        if ((int)subset.size() > begin) {
            plan.group_kind[plan.ngroups] = kind;
            plan.group_begin[plan.ngroups] = begin;
            plan.group_size[plan.ngroups] = (int)subset.size() - begin;
            plan.ngroups++;
        }
    }
    const LaunchShape shape = m0->shape;
    // persistent launch: the work items of every map, stage after stage; the
    // planning, bucketing and leaf-tile items of the batch are shared between
    // the maps in proportion to their walk blocks (so the item list, like the
    // graph, depends only on the walk grid, the variants and the shape)
    std::vector<uint4> items;
    if (shape.persistent) {
        std::vector<uint32_t> cnt((size_t)nmaps * kPersistStages, 0u);
        const long long wtot = start[nmaps];
        const uint32_t leaf_cap = (uint32_t)m0->cus * kMaxLeafBlocksPerCu;
        auto share = [&](int total, int i, uint32_t cap) {
            const long long wb = start[i + 1] - start[i];
            const long long c = ((long long)total * wb + wtot - 1) / wtot;
            return (uint32_t)std::max<long long>(1, std::min<long long>(c, cap));
        };
        for (int i = 0; i < nmaps; ++i) {
            uint32_t *c = &cnt[(size_t)i * kPersistStages];
            const int wb = start[i + 1] - start[i];
            c[0] = (uint32_t)((wb + shape.walk_chunk - 1) / shape.walk_chunk);
            c[1] = share(shape.plan_blocks, i, 0xFFFFu);
            c[2] = share(shape.bucket_blocks, i, 0xFFFFu);
            c[3] = share(shape.leaf_blocks, i, leaf_cap);
            c[4] = voxel_combine_arg(kinds[i]) != -2 ? share(shape.leaf_blocks, i, 0xFFFFu) : 0u;
            c[5] = 1;
            // the commit sums the statistics of this many leaf-tile items
            mds[i].leaf_blocks = (int)c[3];
        }
        for (int st = 0; st < kPersistStages; ++st)
            for (int i = 0; i < nmaps; ++i) {
                const uint32_t *c = &cnt[(size_t)i * kPersistStages];
                int dep = st - 1;
                while (dep >= 0 && c[dep] == 0) --dep;
                const uint32_t w = dep < 0 ? kPersistNoDep
                                           : (uint32_t)(i * kPersistStages + dep) | (c[dep] << 16);
                const uint32_t x = (uint32_t)i | ((uint32_t)st << 16) | ((uint32_t)kinds[i] << 24);
                const uint32_t wb = (uint32_t)(start[i + 1] - start[i]);
                for (uint32_t j = 0; j < c[st]; ++j) {
                    if (st == 0) {
                        const uint32_t b0 = j * (uint32_t)shape.walk_chunk;
                        items.push_back(make_uint4(x, b0, std::min<uint32_t>(shape.walk_chunk, wb - b0), w));
                    } else {
                        items.push_back(make_uint4(x, j, c[st], w));
                    }
                }
            }
    }
    const uint32_t nitems = (uint32_t)items.size();
    const size_t nctl = shape.persistent ? (size_t)kPersistCtlDone + (size_t)nmaps * kPersistStages : 0;
    // per-stage launches: each stage's grid is shared between its maps in
    // proportion to their walk blocks, at least one block each (map q of a
    // launch of P blocks over n maps starts at q + floor(W_q (P - n) / W),
    // W_q the walk blocks of the maps before it)
    std::vector<int> plan_first, bucket_first, part;
    if (!shape.persistent) {
        auto share = [&](const int *maps, int n, int P, std::vector<int> &out) {
            long long W = 0;
            for (int q = 0; q < n; ++q) W += start[maps[q] + 1] - start[maps[q]];
            long long cum = 0;
            for (int q = 0; q <= n; ++q) {
                out.push_back(q + (int)(W > 0 ? cum * (P - n) / W : 0));
                if (q < n) cum += start[maps[q] + 1] - start[maps[q]];
            }
        };
        std::vector<int> all(nmaps);
        for (int i = 0; i < nmaps; ++i) all[i] = i;
        plan.plan_blocks = std::max(shape.plan_blocks, nmaps);
        plan.bucket_blocks = std::max(shape.bucket_blocks, nmaps);
        share(all.data(), nmaps, plan.plan_blocks, plan_first);
        share(all.data(), nmaps, plan.bucket_blocks, bucket_first);
        for (int g = 0; g < plan.ngroups; ++g) {
            const int *gm = subset.data() + plan.group_begin[g];
            const int gs = plan.group_size[g];
            plan.leaf_blocks[g] = std::max(shape.leaf_blocks, gs);
            plan.leaf_part[g] = (int)part.size();
            share(gm, gs, plan.leaf_blocks[g], part);
            // the commit sums the statistics of the map's share of leaf blocks
            for (int q = 0; q < gs; ++q)
                mds[gm[q]].leaf_blocks = part[plan.leaf_part[g] + q + 1] - part[plan.leaf_part[g] + q];
            plan.comb_part[g] = (int)part.size();
            plan.comb_blocks[g] = 0;
            if (voxel_combine_arg(plan.group_kind[g]) != -2) {
                plan.comb_blocks[g] = std::max(combine_blocks(plan.group_kind[g], shape), gs);
                share(gm, gs, plan.comb_blocks[g], part);
            }
        }
    }
    // descriptor: [MapDev x n][FrameParams x n][walk_start x n+1][subset x n]
    // [plan shares][bucket shares][leaf and combine shares][work items]
    // [control block, zero], 16-byte aligned pieces
    auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
    const size_t o_fp = al(sizeof(MapDev) * nmaps), o_ws = o_fp + al(sizeof(FrameParams) * nmaps);
    const size_t o_sub = o_ws + al(sizeof(int) * (nmaps + 1)), o_pf = o_sub + al(sizeof(int) * nmaps);
    const size_t o_bf = o_pf + al(sizeof(int) * plan_first.size());
    const size_t o_pt = o_bf + al(sizeof(int) * bucket_first.size());
    const size_t o_it = o_pt + al(sizeof(int) * part.size());
    const size_t o_ctl = o_it + al(sizeof(uint4) * nitems), bytes = o_ctl + al(sizeof(uint32_t) * nctl);

    if (!m0->batch) m0->batch = new BatchCtx();
    BatchCtx *b = m0->batch;
    if (b->pending) {
        HIP_OK(hipEventSynchronize(b->copied));
        b->pending = false;
    }
    if (bytes > b->cap) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        b->sig.clear();
        if (b->dev) (void)hipFree(b->dev);
        if (b->staging) (void)hipHostFree(b->staging);
        b->dev = nullptr;
        b->staging = nullptr;
        b->cap = 0;
        HIP_OK(hipMalloc(&b->dev, bytes));
        HIP_OK(hipHostMalloc(&b->staging, bytes, hipHostMallocDefault));
        b->cap = bytes;
    }
    if (!b->copied) HIP_OK(hipEventCreateWithFlags(&b->copied, hipEventDisableTiming));
    char *st = (char *)b->staging;
    memcpy(st, mds.data(), sizeof(MapDev) * nmaps);
    memcpy(st + o_fp, fps.data(), sizeof(FrameParams) * nmaps);
    memcpy(st + o_ws, start.data(), sizeof(int) * (nmaps + 1));
    memcpy(st + o_sub, subset.data(), sizeof(int) * nmaps);
    if (!plan_first.empty()) memcpy(st + o_pf, plan_first.data(), sizeof(int) * plan_first.size());
    if (!bucket_first.empty()) memcpy(st + o_bf, bucket_first.data(), sizeof(int) * bucket_first.size());
    if (!part.empty()) memcpy(st + o_pt, part.data(), sizeof(int) * part.size());
    if (nitems) memcpy(st + o_it, items.data(), sizeof(uint4) * nitems);
    if (nctl) memset(st + o_ctl, 0, sizeof(uint32_t) * nctl);
    char *dv = (char *)b->dev;
    MapBatch mb;
    mb.mds = (const MapDev *)dv;
    mb.fps = (const FrameParams *)(dv + o_fp);
    mb.walk_start = (const int *)(dv + o_ws);
    mb.subset = (const int *)(dv + o_sub);
    mb.plan_first = (const int *)(dv + o_pf);
    mb.bucket_first = (const int *)(dv + o_bf);
    mb.part_first = (const int *)(dv + o_pt);
    mb.nmaps = nmaps;
    mb.nsubset = nmaps;
    PersistArgs pa;
    pa.mds = mb.mds;
    pa.fps = mb.fps;
    pa.items = (const uint4 *)(dv + o_it);
    pa.ctl = (uint32_t *)(dv + o_ctl);
    pa.nitems = nitems;
    if (shape.persistent && !b->persist_blocks) b->persist_blocks = persistent_blocks_per_cu() * m0->cus;
    // the control block is zeroed by the descriptor copy itself (no memset in the graph)
    auto launch = [&](hipStream_t q) {
        return shape.persistent ? launch_integrate_persistent(pa, b->persist_blocks, q)
                                : launch_integrate_batched(mb, plan, shape, q);
    };

    if (!use_graph) {
        HIP_OK(hipMemcpyAsync(b->dev, b->staging, bytes, hipMemcpyHostToDevice, s));
        HIP_OK(launch(s));
    } else {
        // the graph holds grid sizes, the grouping and the item count;
        // everything else is read from the descriptor, which the graph copies
        // in at each replay
        std::vector<long long> sig = {nmaps, (long long)bytes, shape.plan_blocks, shape.bucket_blocks,
                                      shape.leaf_blocks, shape.persistent, shape.walk_chunk, shape.wave_pairs,
                                      shape.slab_pairs, nitems};
        for (int i = 0; i <= nmaps; ++i) sig.push_back(start[i]);
        for (int i = 0; i < nmaps; ++i) sig.push_back(kinds[i]);
        if (sig != b->sig || !b->exec) {
            if (b->exec) (void)hipGraphExecDestroy(b->exec);
            if (b->graph) (void)hipGraphDestroy(b->graph);
            b->exec = nullptr;
            b->graph = nullptr;
            b->sig.clear();
            if (!b->cap_stream) HIP_OK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
            HIP_OK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e1 = hipMemcpyAsync(b->dev, b->staging, bytes, hipMemcpyHostToDevice, b->cap_stream);
            hipError_t e2 = launch(b->cap_stream);
            hipGraph_t graph = nullptr;
            hipError_t e3 = hipStreamEndCapture(b->cap_stream, &graph);
            if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(SLIM_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e1 ? e1 : (e2 ? e2 : e3)));
            }
            b->graph = graph;
            HIP_OK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            b->sig = sig;
        }
        HIP_OK(hipGraphLaunch(b->exec, s));
    }
    HIP_OK(hipEventRecord(b->copied, s));
    b->pending = true;
    return SLIM_OK;
}

slim_status slim_profile_enable(slim_map *m, int32_t enable)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    DeviceGuard g(m->cfg.device);
    if (enable && m->ev.empty()) {
        m->ev.resize((size_t)kProfRing * 2 * kNumProfiled);
        // device-scope release: the stage brackets time the kernels, not
        // system-scope cache writebacks
        for (auto &e : m->ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventReleaseToDevice));
    }
    m->prof = enable != 0;
    return SLIM_OK;
}

slim_status slim_profile_read(slim_map *m, double *ms, int64_t *launches, int32_t n_kernels, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (n_kernels < 0 || (n_kernels > 0 && (!ms || !launches))) return fail(SLIM_ERR_INVALID, "bad output arrays");
    DeviceGuard g(m->cfg.device);
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    slim_status r = drain_profile(m, true);
    if (r) return r;
    for (int k = 0; k < std::min(n_kernels, kNumProfiled); ++k) {
        ms[k] = m->prof_ms[k];
        launches[k] = m->prof_n[k];
        m->prof_ms[k] = 0.0;
        m->prof_n[k] = 0;
    }
    return SLIM_OK;
}

slim_status slim_profile_sets(slim_map *m, int32_t capacity, int32_t *frames, double *ms, double *span_ms,
                              int32_t *count, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (!count || capacity < 0 || (capacity > 0 && (!frames || !ms || !span_ms)))
        return fail(SLIM_ERR_INVALID, "bad output arrays");
    DeviceGuard g(m->cfg.device);
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    slim_status r = drain_profile(m, true);
    if (r) return r;
    const int n = (int)m->prof_sets.size();
    *count = n;
    for (int i = 0; i < std::min(n, capacity); ++i) {
        const slim_map::ProfSet &ps = m->prof_sets[(size_t)i];
        frames[i] = ps.frames;
        for (int k = 0; k < kNumProfiled; ++k) ms[(size_t)i * kNumProfiled + k] = ps.ms[k];
        span_ms[i] = ps.span;
    }
    m->prof_sets.clear();
    return SLIM_OK;
}

}  // extern "C"
