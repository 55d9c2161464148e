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

}  // namespace

struct slim_map {
    slim_map_config cfg;
    int nsem = 0;
    int maxsteps = 0;
    int cus = 256;
    MapDev md = {};
    size_t hcap = 0;
    size_t pair_cap = 0;
    // extraction scratch
    unsigned long long *ext_keys = nullptr;
    int32_t *ext_slots = nullptr;
    uint32_t *ext_offsets = nullptr;
    size_t ext_cap = 0;
    // kernel timing
    bool prof = false;
    std::vector<hipEvent_t> ev;  // kProfRing * 2 * kNumProfiled
    int prof_head = 0, prof_count = 0;
    double prof_ms[kNumProfiled] = {};
    long long prof_n[kNumProfiled] = {};
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

void free_all(slim_map *m)
{
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
    if ((double)c->max_range / (double)c->voxel_size >= (double)(1 << 19))
        return fail(SLIM_ERR_INVALID, "max_range must be below 2^19 voxel sizes");
    if (c->sem_mode == SLIM_SEM_CLOSED) {
        if (c->num_classes < 1 || c->num_classes > 256) return fail(SLIM_ERR_INVALID, "num_classes must be 1..256");
    } else if (c->sem_mode == SLIM_SEM_OPEN) {
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

slim_status ensure_pairs(slim_map *m, size_t need, hipStream_t s)
{
    if (need <= m->pair_cap) return SLIM_OK;
    if (need > 0xFFFFFFF0ull) return fail(SLIM_ERR_INVALID, "frame needs more than 2^32 pair slots");
    HIP_OK(hipStreamSynchronize(s));
    size_t cap = std::max<size_t>(need, m->pair_cap + m->pair_cap / 2);
    cap = std::min<size_t>(cap, 0xFFFFFFF0ull);
    MapDev &md = m->md;
    void *ptrs[8] = {md.pair_pos, md.pair_rank, md.pair_key, md.pair_tsdf,
                     md.srt_key,  md.srt_tsdf,  md.tmp_key,  md.tmp_tsdf};
    for (void *p : ptrs) {
        if (!p) continue;
        (void)hipFree(p);
        m->allocs.erase(std::remove(m->allocs.begin(), m->allocs.end(), p), m->allocs.end());
    }
    md.pair_pos = md.pair_rank = md.pair_key = md.srt_key = md.tmp_key = nullptr;
    md.pair_tsdf = md.srt_tsdf = md.tmp_tsdf = nullptr;
    slim_status r;
    if ((r = dalloc(m, &md.pair_pos, cap)) || (r = dalloc(m, &md.pair_rank, cap)) ||
        (r = dalloc(m, &md.pair_key, cap)) || (r = dalloc(m, &md.pair_tsdf, cap)) ||
        (r = dalloc(m, &md.srt_key, cap)) || (r = dalloc(m, &md.srt_tsdf, cap)) ||
        (r = dalloc(m, &md.tmp_key, cap)) || (r = dalloc(m, &md.tmp_tsdf, cap))) {
        m->pair_cap = 0;
        md.pair_cap = 0;
        return r;
    }
    m->pair_cap = cap;
    md.pair_cap = (uint32_t)cap;
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
        for (int k = 0; k < kNumProfiled; ++k) {
            float ms = 0.0f;
            HIP_OK(hipEventElapsedTime(&ms, e[2 * k], e[2 * k + 1]));
            m->prof_ms[k] += ms;
            m->prof_n[k] += 1;
        }
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
    m->nsem = config->sem_mode == SLIM_SEM_CLOSED ? config->num_classes
              : config->sem_mode == SLIM_SEM_OPEN ? 2 * config->embed_dim
                                                   : 0;
    m->maxsteps = max_steps(config->voxel_size, config->sdf_trunc);
    size_t cap = 1024;
    while (cap < 2 * (size_t)config->max_leaves) cap <<= 1;
    m->hcap = cap;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, config->device) == hipSuccess && prop.multiProcessorCount > 0)
        m->cus = prop.multiProcessorCount;

    MapDev &md = m->md;
    md.hmask = (uint32_t)(cap - 1);
    md.max_leaves = config->max_leaves;
    md.max_pages = (config->max_voxels + kPageVoxels - 1) / kPageVoxels;
    md.rec_stride = record_stride(m->nsem);
    md.leaf_blocks = m->cus * 8;
    const size_t L = (size_t)config->max_leaves, NP = (size_t)md.max_pages;
    if ((r = dalloc(m, &md.hkeys, cap)) || (r = dalloc(m, &md.hvals, cap)) || (r = dalloc(m, &md.skeys, cap)) ||
        (r = dalloc(m, &md.touched, cap)) || (r = dalloc(m, &md.pos_count, cap)) ||
        (r = dalloc(m, &md.pos_slab, cap)) || (r = dalloc(m, &md.pos_plan, cap)) ||
        (r = dalloc(m, &md.pos_pages, 2 * cap)) || (r = dalloc(m, &md.leaf_key, L)) ||
        (r = dalloc(m, &md.leaf_page, L * kLeafPages)) || (r = dalloc(m, &md.leaf_occ, L * kMaskWords)) ||
        (r = dalloc(m, &md.vox, NP * kPageVoxels * (size_t)md.rec_stride)) ||
        (r = dalloc(m, &md.blk_stats, (size_t)md.leaf_blocks)) || (r = dalloc(m, &md.st, 1))) {
        free_all(m);
        delete m;
        return r;
    }
    if (launch_reset(md, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        free_all(m);
        delete m;
        return fail(SLIM_ERR_DEVICE, "map initialisation failed");
    }
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
    return SLIM_OK;
}

slim_status slim_integrate(slim_map *m, const float *points, int64_t n, const double *pose, const void *sem,
                           int32_t kind, void *stream)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    if (n < 0 || n >= kMaxPoints) return fail(SLIM_ERR_INVALID, "n must be in [0, 2^23)");
    if (n > 0 && !points) return fail(SLIM_ERR_INVALID, "points is NULL");
    if (((uintptr_t)points & 3u) != 0) return fail(SLIM_ERR_INVALID, "points must be 4-byte aligned");
    if (!pose) return fail(SLIM_ERR_INVALID, "pose is NULL");
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(pose[i])) return fail(SLIM_ERR_INVALID, "pose has a non-finite entry");
    const slim_map_config &c = m->cfg;
    bool kind_ok = false;
    if (c.sem_mode == SLIM_SEM_NONE) kind_ok = kind == SLIM_IN_NONE;
    if (c.sem_mode == SLIM_SEM_CLOSED)
        kind_ok = kind == SLIM_IN_LABEL_I32 || kind == SLIM_IN_PROB_F32 || kind == SLIM_IN_LOGIT_F32;
    if (c.sem_mode == SLIM_SEM_OPEN) kind_ok = kind == SLIM_IN_EMB_BF16 || kind == SLIM_IN_EMB_F32;
    if (!kind_ok) return fail(SLIM_ERR_INVALID, "semantic input kind %d does not match the map's mode", kind);
    if (kind == SLIM_IN_LOGIT_F32 && c.num_classes > 64)
        return fail(SLIM_ERR_UNSUPPORTED, "logit input supports at most 64 classes");
    if (kind != SLIM_IN_NONE && n > 0 && !sem) return fail(SLIM_ERR_INVALID, "semantic input is NULL");
    if (((uintptr_t)sem & (kind == SLIM_IN_EMB_BF16 ? 1u : 3u)) != 0)
        return fail(SLIM_ERR_INVALID, "semantic input is misaligned");

    FrameParams fp;
    const double vsd = (double)c.voxel_size;
    for (int r = 0; r < 3; ++r) {
        const double ta = pose[4 * r + 3];
        const double q = std::floor(ta / vsd);
        if (!(std::fabs(q) < (double)(1 << 19)))
            return fail(SLIM_ERR_INVALID, "pose translation beyond 2^19 voxel sizes");
        fp.a[r] = (int)q;
        fp.t[r] = (float)(ta - (double)fp.a[r] * vsd);
        for (int k = 0; k < 3; ++k) fp.R[3 * r + k] = (float)pose[4 * r + k];
    }
    fp.vs = c.voxel_size;
    fp.tau = c.sdf_trunc;
    fp.rmin = c.min_range;
    fp.rmax = c.max_range;
    fp.maxsteps = m->maxsteps;
    fp.n = (int)n;
    fp.sem_kind = kind;
    fp.K = c.sem_mode == SLIM_SEM_CLOSED ? c.num_classes : 0;
    fp.L = c.sem_mode == SLIM_SEM_OPEN ? c.embed_dim : 0;
    fp.nsem = m->nsem;
    fp.pts = points;
    fp.sem = sem;

    DeviceGuard g(c.device);
    hipStream_t s = (hipStream_t)stream;
    slim_status r = ensure_pairs(m, (size_t)std::max<int64_t>(n, 1) * (size_t)m->maxsteps, s);
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
        m->prof_head = (m->prof_head + 1) % kProfRing;
        m->prof_count++;
    }
    HIP_OK(launch_integrate(fp, m->md, m->cus, s, ev));
    return SLIM_OK;
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

slim_status slim_profile_enable(slim_map *m, int32_t enable)
{
    g_err[0] = 0;
    if (!m) return fail(SLIM_ERR_INVALID, "map is NULL");
    DeviceGuard g(m->cfg.device);
    if (enable && m->ev.empty()) {
        m->ev.resize((size_t)kProfRing * 2 * kNumProfiled);
        for (auto &e : m->ev) HIP_OK(hipEventCreate(&e));
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

}  // extern "C"
