/*
 * slim_oracle.c -- plain, slow, FP64 CPU oracle for the per-frame fused TSDF +
 * Bayesian semantic integration of SLIM-VDB (arXiv 2512.12945).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path; the two meet only in the seeded synthetic inputs.
 *
 * What it computes (paper, Sec. III-A to III-D):
 *   - for every point of a posed cloud, the voxels of the truncation band
 *     around the point along its sensor ray (Sec. III-A, "configurable
 *     truncated region"), visited with an Amanatides-Woo voxel walk;
 *   - per visited voxel the projective signed distance, truncated (Sec. III-A,
 *     Curless-Levoy);
 *   - the running TSDF mean and weight, Eq. (1)-(2), with weight 1;
 *   - closed set: Dirichlet concentration update, Thm. 1 / Eq. (6);
 *   - open set: Normal-Inverse-Gamma update, Thm. 2 / Eqs. (11)-(14), with
 *     lambda = 2 nu = W and a diagonal beta (Sec. III-D, implementation note).
 *
 * Precision: the geometric *decision* path (pose application, ray, band, voxel
 * walk, truncation gate) is a fixed sequence of IEEE binary32 operations, so
 * that an independent FP32 implementation can reproduce the same voxel keys
 * bit for bit.  Every accumulated *value* (signed distance, weights, class
 * counts, embedding statistics) is FP64.  Build with -ffp-contract=off and
 * without fast-math: only the fmaf() calls written below fuse.
 *
 * Each frame is applied as one batch per voxel (Thm. 1 and Thm. 2 are stated
 * for a set of observations), or, in sequential mode, one observation at a
 * time in point order (the paper's per-point recursion).  Both are exposed so
 * that the tests can check they agree.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- input kinds (values shared with the Python wrapper by convention) ---- */
/* CLOSED_LAST and OPEN_LAST: the non-Bayesian ablation of Sec. IV (SLIM-VDB*),
 * where a voxel's semantics are those of its most recent measurement. */
enum { OM_SEM_NONE = 0, OM_SEM_CLOSED = 1, OM_SEM_OPEN = 2, OM_SEM_CLOSED_LAST = 3, OM_SEM_OPEN_LAST = 4 };
enum { OM_IN_NONE = 0, OM_IN_LABEL_I32 = 1, OM_IN_PROB_F32 = 2, OM_IN_LOGIT_F32 = 3,
       OM_IN_EMB_BF16 = 4, OM_IN_EMB_F32 = 5 };

#define OM_KEY_LIMIT (1 << 20) /* a voxel coordinate must satisfy |k| < 2^20 */
#define OM_EMPTY UINT64_MAX

typedef struct {
    /* parameters, as the float values the caller configured */
    float vs, tau, rmin, rmax;
    int sem_mode, K, L, nsem; /* nsem: K (closed), 2L (open: m then beta), 1 (closed last: class),
                                 L (open last: embedding), 0 */
    int maxsteps;
    /* voxel table: packed key -> record */
    uint64_t *hkey;
    int64_t *hval;
    int64_t hcap, hused;
    /* records */
    int64_t nvox, vcap;
    uint64_t *vkey;
    double *D, *W, *sem;
    /* leaf table (set of leaf keys) */
    uint64_t *lkey;
    int64_t lcap, nleaf;
    /* counters of the last frame */
    int64_t st_points, st_rejected, st_pairs, st_uold, st_unew, st_newleaf;
} omap;

/* ------------------------------------------------------------------------- */
/* small helpers                                                             */
/* ------------------------------------------------------------------------- */

static uint64_t mix64(uint64_t x)
{
    x ^= x >> 30; x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27; x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

/* three signed coordinates, |c| < 2^20, packed as biased 21-bit fields */
static uint64_t pack3(int32_t x, int32_t y, int32_t z)
{
    return ((uint64_t)(uint32_t)(x + OM_KEY_LIMIT) << 42) |
           ((uint64_t)(uint32_t)(y + OM_KEY_LIMIT) << 21) |
           (uint64_t)(uint32_t)(z + OM_KEY_LIMIT);
}

static void unpack3(uint64_t k, int32_t c[3])
{
    c[0] = (int32_t)((k >> 42) & 0x1FFFFF) - OM_KEY_LIMIT;
    c[1] = (int32_t)((k >> 21) & 0x1FFFFF) - OM_KEY_LIMIT;
    c[2] = (int32_t)(k & 0x1FFFFF) - OM_KEY_LIMIT;
}

/* floor division by 8, written without relying on signed shifts */
static int32_t floor_div8(int32_t v) { return v >= 0 ? v / 8 : -((-v + 7) / 8); }

static double bf16_to_double(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* ------------------------------------------------------------------------- */
/* map storage: open-addressing table of voxel records, FP64 fields          */
/* ------------------------------------------------------------------------- */

static int table_grow(uint64_t **keys, int64_t **vals, int64_t *cap)
{
    int64_t ncap = *cap ? *cap * 2 : 1024;
    uint64_t *nk = (uint64_t *)malloc((size_t)ncap * sizeof(uint64_t));
    int64_t *nv = vals ? (int64_t *)malloc((size_t)ncap * sizeof(int64_t)) : NULL;
    if (!nk || (vals && !nv)) { free(nk); free(nv); return -1; }
    for (int64_t i = 0; i < ncap; ++i) nk[i] = OM_EMPTY;
    for (int64_t i = 0; i < *cap; ++i) {
        uint64_t k = (*keys)[i];
        if (k == OM_EMPTY) continue;
        int64_t h = (int64_t)(mix64(k) & (uint64_t)(ncap - 1));
        while (nk[h] != OM_EMPTY) h = (h + 1) & (ncap - 1);
        nk[h] = k;
        if (vals) nv[h] = (*vals)[i];
    }
    free(*keys);
    *keys = nk;
    if (vals) { free(*vals); *vals = nv; }
    *cap = ncap;
    return 0;
}

/* returns the table position of k, or -1 if absent */
static int64_t table_find(const uint64_t *keys, int64_t cap, uint64_t k)
{
    if (cap == 0) return -1;
    int64_t h = (int64_t)(mix64(k) & (uint64_t)(cap - 1));
    while (keys[h] != OM_EMPTY) {
        if (keys[h] == k) return h;
        h = (h + 1) & (cap - 1);
    }
    return -1;
}

/* inserts k (known absent); returns its position */
static int64_t table_insert(uint64_t *keys, int64_t cap, uint64_t k)
{
    int64_t h = (int64_t)(mix64(k) & (uint64_t)(cap - 1));
    while (keys[h] != OM_EMPTY) h = (h + 1) & (cap - 1);
    keys[h] = k;
    return h;
}

/* Returns the record of voxel key k, creating a zero record if absent.
 * *created is set to 1 for a new record. Returns -1 on allocation failure. */
static int64_t voxel_get(omap *m, uint64_t k, int *created)
{
    int64_t pos = table_find(m->hkey, m->hcap, k);
    *created = 0;
    if (pos >= 0) return m->hval[pos];
    if (2 * (m->hused + 1) > m->hcap)
        if (table_grow(&m->hkey, &m->hval, &m->hcap)) return -1;
    if (m->nvox == m->vcap) {
        int64_t nc = m->vcap ? m->vcap * 2 : 1024;
        uint64_t *vk = (uint64_t *)realloc(m->vkey, (size_t)nc * sizeof(uint64_t));
        if (!vk) return -1;
        m->vkey = vk;
        double *d = (double *)realloc(m->D, (size_t)nc * sizeof(double));
        if (!d) return -1;
        m->D = d;
        double *w = (double *)realloc(m->W, (size_t)nc * sizeof(double));
        if (!w) return -1;
        m->W = w;
        if (m->nsem) {
            double *s = (double *)realloc(m->sem, (size_t)nc * (size_t)m->nsem * sizeof(double));
            if (!s) return -1;
            m->sem = s;
        }
        m->vcap = nc;
    }
    int64_t r = m->nvox++;
    m->vkey[r] = k;
    m->D[r] = 0.0;
    m->W[r] = 0.0;
    if (m->nsem) memset(m->sem + r * m->nsem, 0, (size_t)m->nsem * sizeof(double));
    pos = table_insert(m->hkey, m->hcap, k);
    m->hval[pos] = r;
    m->hused++;
    *created = 1;

    /* leaf bookkeeping: the 8^3 block containing the voxel */
    int32_t c[3];
    unpack3(k, c);
    uint64_t lk = pack3(floor_div8(c[0]), floor_div8(c[1]), floor_div8(c[2]));
    if (table_find(m->lkey, m->lcap, lk) < 0) {
        if (2 * (m->nleaf + 1) > m->lcap)
            if (table_grow(&m->lkey, NULL, &m->lcap)) return -1;
        table_insert(m->lkey, m->lcap, lk);
        m->nleaf++;
        m->st_newleaf++;
    }
    return r;
}

/* ------------------------------------------------------------------------- */
/* creation                                                                  */
/* ------------------------------------------------------------------------- */

omap *om_create(float vs, float tau, float rmin, float rmax, int sem_mode, int K, int L)
{
    if (!(vs > 0.0f) || !(tau >= vs) || !(rmin >= 0.0f) || !(rmax > rmin)) return NULL;
    if ((sem_mode == OM_SEM_CLOSED || sem_mode == OM_SEM_CLOSED_LAST) && K < 1) return NULL;
    if ((sem_mode == OM_SEM_OPEN || sem_mode == OM_SEM_OPEN_LAST) && L < 1) return NULL;
    if (sem_mode < OM_SEM_NONE || sem_mode > OM_SEM_OPEN_LAST) return NULL;
    omap *m = (omap *)calloc(1, sizeof(omap));
    if (!m) return NULL;
    m->vs = vs; m->tau = tau; m->rmin = rmin; m->rmax = rmax;
    m->sem_mode = sem_mode; m->K = K; m->L = L;
    m->nsem = sem_mode == OM_SEM_CLOSED        ? K
              : sem_mode == OM_SEM_OPEN        ? 2 * L
              : sem_mode == OM_SEM_CLOSED_LAST ? 1
              : sem_mode == OM_SEM_OPEN_LAST   ? L
                                               : 0;
    /* visit cap: the band is at most 2 tau long; a walk of that length crosses
     * at most 2 tau / vs planes per axis plus one; this bound is generous. */
    m->maxsteps = 3 * (int)ceil((2.0 * (double)tau) / (double)vs) + 4;
    return m;
}

void om_destroy(omap *m)
{
    if (!m) return;
    free(m->hkey); free(m->hval); free(m->vkey); free(m->D); free(m->W); free(m->sem);
    free(m->lkey);
    free(m);
}

int om_maxsteps(const omap *m) { return m->maxsteps; }

/* ------------------------------------------------------------------------- */
/* geometric decision path (binary32, fixed operation order)                 */
/* ------------------------------------------------------------------------- */

typedef struct {
    float R[9];     /* rotation, rounded to binary32 */
    float t[3];     /* sensor origin relative to the anchor voxel corner */
    int32_t a[3];   /* anchor voxel */
} oframe;

/* The pose is map_T_sensor, 4x4 row-major, FP64.  The anchor is the voxel that
 * holds the sensor origin; all FP32 geometry is done relative to its corner so
 * that coordinates stay small whatever the map extent. */
static void frame_setup(const omap *m, const double P[16], oframe *f)
{
    double vsd = (double)m->vs;
    for (int r = 0; r < 3; ++r) {
        double ta = P[r * 4 + 3];
        double q = floor(ta / vsd);
        if (!(fabs(q) < (double)OM_KEY_LIMIT)) q = (double)OM_KEY_LIMIT; /* rejected later */
        f->a[r] = (int32_t)q;
        f->t[r] = (float)(ta - (double)f->a[r] * vsd);
        for (int c = 0; c < 3; ++c) f->R[r * 3 + c] = (float)P[r * 4 + c];
    }
}

/* Amanatides-Woo walk over the band [t0, t1] of the ray o + t u.  Writes the
 * visited cells (relative to the anchor) and returns how many were visited. */
static int band_walk(float vs, int maxsteps, const float o[3], const float u[3], float t0, float t1,
                     int32_t (*cells)[3])
{
    int32_t c[3], step[3];
    float tmax[3], tdel[3];
    for (int a = 0; a < 3; ++a) {
        float s = fmaf(t0, u[a], o[a]);
        float fc = floorf(s / vs);
        /* a start cell 2^30 or more cells out is far outside the key range;
         * it is held there (no integer overflow) and the point is rejected */
        if (!(fabsf(fc) < 1073741824.0f)) fc = fc < 0.0f ? -1073741824.0f : 1073741824.0f;
        c[a] = (int32_t)fc;
        if (u[a] > 0.0f) {
            step[a] = 1;
            tmax[a] = t0 + fmaf((float)(c[a] + 1), vs, -s) / u[a];
            tdel[a] = vs / u[a];
        } else if (u[a] < 0.0f) {
            step[a] = -1;
            tmax[a] = t0 + fmaf((float)c[a], vs, -s) / u[a];
            tdel[a] = -vs / u[a];
        } else {
            step[a] = 0;
            tmax[a] = INFINITY;
            tdel[a] = INFINITY;
        }
    }
    int nv = 0;
    for (int it = 0; it < maxsteps; ++it) {
        cells[nv][0] = c[0]; cells[nv][1] = c[1]; cells[nv][2] = c[2];
        nv++;
        /* axis of the nearest boundary; ties go to the lowest axis */
        int ax;
        if (tmax[0] <= tmax[1]) ax = (tmax[0] <= tmax[2]) ? 0 : 2;
        else ax = (tmax[1] <= tmax[2]) ? 1 : 2;
        if (tmax[ax] > t1) break;
        c[ax] += step[ax];
        tmax[ax] += tdel[ax];
    }
    return nv;
}

/* Ray of one sensor-frame point.  Returns 1 and fills p (point), u (unit
 * direction), r (range) if the point passes the validity and range gates. */
static int point_ray(const omap *m, const oframe *f, const float ps[3], float p[3], float u[3], float *r)
{
    if (!isfinite(ps[0]) || !isfinite(ps[1]) || !isfinite(ps[2])) return 0;
    for (int a = 0; a < 3; ++a)
        p[a] = fmaf(f->R[a * 3 + 0], ps[0], fmaf(f->R[a * 3 + 1], ps[1], fmaf(f->R[a * 3 + 2], ps[2], f->t[a])));
    float d[3] = {p[0] - f->t[0], p[1] - f->t[1], p[2] - f->t[2]};
    float rr = sqrtf(fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0])));
    if (!(rr > 0.0f) || !isfinite(rr) || rr < m->rmin || rr > m->rmax) return 0;
    for (int a = 0; a < 3; ++a) u[a] = d[a] / rr;
    *r = rr;
    return 1;
}

/* Signed distance of the voxel centre to the point along the ray: positive in
 * front of the surface.  sdf32 (decision) in the fixed FP32 form; the value
 * is the same quantity in FP64 from the FP32 inputs. */
static float sdf_decision(float vs, const int32_t c[3], const float p[3], const float u[3])
{
    float q[3];
    for (int a = 0; a < 3; ++a) q[a] = fmaf(-(float)c[a], vs, p[a]) - 0.5f * vs;
    return fmaf(q[2], u[2], fmaf(q[1], u[1], q[0] * u[0]));
}

static double sdf_value(float vs, const int32_t c[3], const float p[3], const float u[3])
{
    double s = 0.0;
    for (int a = 0; a < 3; ++a)
        s += ((double)p[a] - ((double)c[a] + 0.5) * (double)vs) * (double)u[a];
    return s;
}

/* ------------------------------------------------------------------------- */
/* per-frame observation pairs                                               */
/* ------------------------------------------------------------------------- */

/* Cells visited by the band walk of one ray, before the truncation gate (for
 * checking the walk itself).  o, p are FP32 coordinates in voxel-size units
 * of the given vs.  Returns the number of cells (<= cap). */
int om_ray_visits(float vs, float tau, const float o[3], const float p[3], int32_t *cells, int cap)
{
    int maxsteps = 3 * (int)ceil((2.0 * (double)tau) / (double)vs) + 4;
    float d[3] = {p[0] - o[0], p[1] - o[1], p[2] - o[2]};
    float r = sqrtf(fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0])));
    if (!(r > 0.0f)) return 0;
    float u[3] = {d[0] / r, d[1] / r, d[2] / r};
    float t0 = fmaxf(r - tau, 0.0f), t1 = r + tau;
    int32_t(*tmp)[3] = (int32_t(*)[3])malloc((size_t)maxsteps * sizeof(*tmp));
    int nv = band_walk(vs, maxsteps, o, u, t0, t1, tmp);
    if (nv > cap) nv = cap;
    memcpy(cells, tmp, (size_t)nv * sizeof(*tmp));
    free(tmp);
    return nv;
}

static int label_ok(const omap *m, const void *sem, int kind, int64_t j)
{
    if ((m->sem_mode == OM_SEM_CLOSED || m->sem_mode == OM_SEM_CLOSED_LAST) && kind == OM_IN_LABEL_I32) {
        int32_t l = ((const int32_t *)sem)[j];
        return l >= 0 && l < m->K;
    }
    return 1;
}

/* Back-projects a depth image (row-major height x width, metres along the
 * optical axis) through pinhole intrinsics into sensor-frame points, point
 * i = v * width + u: x = ((u - cx) / fx) d, y = ((v - cy) / fy) d, z = d, each
 * operation rounded to binary32 in that order (the RGB-D input of Sec. III-A,
 * an image turned into points).  A depth that is not finite and > 0 gives a NaN
 * point, which integration rejects. */
void om_depth_points(const float *depth, int width, int height, float fx, float fy, float cx, float cy,
                     float *pts)
{
    for (int v = 0; v < height; ++v)
        for (int u = 0; u < width; ++u) {
            int64_t i = (int64_t)v * width + u;
            float d = depth[i];
            float *p = pts + 3 * i;
            if (!(d > 0.0f) || !isfinite(d)) {
                p[0] = p[1] = p[2] = NAN;
                continue;
            }
            float xr = ((float)u - cx) / fx, yr = ((float)v - cy) / fy;
            p[0] = xr * d;
            p[1] = yr * d;
            p[2] = d;
        }
}

/* Enumerates the observation pairs of one frame: every (voxel, point) where
 * the voxel lies on the point's band walk and passes the gate sdf > -tau.
 * keys: P x 3 absolute voxel coordinates; pid: point index; tsdf: min(sdf,
 * tau) in FP64; sdf32: the FP32 decision value.  A point is rejected (and
 * contributes nothing) if it is non-finite, outside [rmin, rmax], has an
 * invalid label, or if any visited voxel falls outside |k| < 2^20.
 * Returns the pair count; if it exceeds cap, nothing beyond cap is written
 * and the full count is still returned. */
int64_t om_frame_pairs(const omap *m, const float *pts, int64_t n, const double pose[16], const void *sem,
                       int kind, int32_t *keys, uint32_t *pid, double *tsdf, float *sdf32, int64_t cap,
                       int64_t *rejected)
{
    oframe f;
    frame_setup(m, pose, &f);
    int32_t(*cells)[3] = (int32_t(*)[3])malloc((size_t)m->maxsteps * sizeof(*cells));
    int64_t np = 0, nrej = 0;
    for (int64_t j = 0; j < n; ++j) {
        float p[3], u[3], r;
        if (!point_ray(m, &f, pts + 3 * j, p, u, &r) || !label_ok(m, sem, kind, j)) { nrej++; continue; }
        float t0 = fmaxf(r - m->tau, 0.0f), t1 = r + m->tau;
        int nv = band_walk(m->vs, m->maxsteps, f.t, u, t0, t1, cells);
        int inrange = 1;
        for (int i = 0; i < nv; ++i)
            for (int a = 0; a < 3; ++a) {
                int64_t k = (int64_t)f.a[a] + cells[i][a];
                if (!(k > -OM_KEY_LIMIT && k < OM_KEY_LIMIT)) inrange = 0;
            }
        if (!inrange) { nrej++; continue; }
        for (int i = 0; i < nv; ++i) {
            float s32 = sdf_decision(m->vs, cells[i], p, u);
            if (!(s32 > -m->tau)) continue;
            if (np < cap) {
                for (int a = 0; a < 3; ++a) keys[3 * np + a] = f.a[a] + cells[i][a];
                pid[np] = (uint32_t)j;
                double s = sdf_value(m->vs, cells[i], p, u);
                tsdf[np] = s < (double)m->tau ? s : (double)m->tau;
                sdf32[np] = s32;
            }
            np++;
        }
    }
    free(cells);
    if (rejected) *rejected = nrej;
    return np;
}

/* ------------------------------------------------------------------------- */
/* conjugate combine                                                         */
/* ------------------------------------------------------------------------- */

/* The weight row of one observation (Sec. III-C/D): closed set -> a vector of
 * K class weights summing to 1 (one-hot label, given probabilities, or the
 * softmax of logits); open set -> the L-dim embedding. */
static void sem_row(const omap *m, const void *sem, int kind, int64_t j, double *out)
{
    if (m->sem_mode == OM_SEM_CLOSED) {
        int K = m->K;
        if (kind == OM_IN_LABEL_I32) {
            int32_t l = ((const int32_t *)sem)[j];
            for (int i = 0; i < K; ++i) out[i] = (i == l) ? 1.0 : 0.0;
        } else if (kind == OM_IN_PROB_F32) {
            const float *p = (const float *)sem + j * K;
            for (int i = 0; i < K; ++i) out[i] = (double)p[i];
        } else { /* logits: softmax in FP64 */
            const float *l = (const float *)sem + j * K;
            double mx = (double)l[0];
            for (int i = 1; i < K; ++i) if ((double)l[i] > mx) mx = (double)l[i];
            double s = 0.0;
            for (int i = 0; i < K; ++i) { out[i] = exp((double)l[i] - mx); s += out[i]; }
            for (int i = 0; i < K; ++i) out[i] /= s;
        }
    } else if (m->sem_mode == OM_SEM_OPEN || m->sem_mode == OM_SEM_OPEN_LAST) {
        int L = m->L;
        if (kind == OM_IN_EMB_BF16) {
            const uint16_t *z = (const uint16_t *)sem + j * L;
            for (int d = 0; d < L; ++d) out[d] = bf16_to_double(z[d]);
        } else {
            const float *z = (const float *)sem + j * L;
            for (int d = 0; d < L; ++d) out[d] = (double)z[d];
        }
    }
}

/* The class a single measurement names (non-Bayesian mode): the label, or the
 * first index of the largest given probability or logit.  Compared in the
 * input's own binary32 values. */
static int last_class(const omap *m, const void *sem, int kind, int64_t j)
{
    if (kind == OM_IN_LABEL_I32) return ((const int32_t *)sem)[j];
    const float *row = (const float *)sem + j * m->K;
    int best = 0;
    for (int i = 1; i < m->K; ++i)
        if (row[i] > row[best]) best = i;
    return best;
}

typedef struct { uint64_t key; uint32_t pid; int64_t idx; } opair_ref;

static int cmp_pair(const void *a, const void *b)
{
    const opair_ref *x = (const opair_ref *)a, *y = (const opair_ref *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->pid != y->pid) return x->pid < y->pid ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Applies P observation pairs to the map.
 * mode 0 (batch): every voxel receives its pairs as one set, Thm. 1 / Thm. 2.
 * mode 1 (sequential): one observation at a time, in (voxel, point) order.
 * sem/kind/npts describe the per-point semantic rows referenced by pid.
 * Returns 0, or -1 on allocation failure. */
int om_apply(omap *m, int64_t P, const int32_t *keys, const uint32_t *pid, const double *tsdf, const void *sem,
             int kind, int mode)
{
    opair_ref *ord = (opair_ref *)malloc((size_t)(P > 0 ? P : 1) * sizeof(opair_ref));
    if (!ord) return -1;
    for (int64_t i = 0; i < P; ++i) {
        ord[i].key = pack3(keys[3 * i], keys[3 * i + 1], keys[3 * i + 2]);
        ord[i].pid = pid[i];
        ord[i].idx = i;
    }
    qsort(ord, (size_t)P, sizeof(opair_ref), cmp_pair);

    int nsem = m->nsem;
    int rowlen = m->sem_mode == OM_SEM_CLOSED ? m->K : (m->sem_mode == OM_SEM_OPEN ? m->L : 0);
    int last = m->sem_mode == OM_SEM_CLOSED_LAST || m->sem_mode == OM_SEM_OPEN_LAST;
    int64_t rowcap = 0;
    double *rows = NULL;     /* rows of the current segment */

    int64_t s = 0;
    while (s < P) {
        int64_t e = s + 1;
        if (mode == 0)
            while (e < P && ord[e].key == ord[s].key) e++;
        int64_t n = e - s;
        int created;
        int64_t r = voxel_get(m, ord[s].key, &created);
        if (r < 0) { free(ord); free(rows); return -1; }
        /* a voxel seen for the first time in this frame counts once */
        if (s == 0 || ord[s - 1].key != ord[s].key) {
            if (created) m->st_unew++;
            else m->st_uold++;
        }

        /* Eq. (1)-(2): weighted running mean with unit weights */
        double sum_t = 0.0;
        for (int64_t i = s; i < e; ++i) sum_t += tsdf[ord[i].idx];
        double W0 = m->W[r], W1 = W0 + (double)n;
        m->D[r] = (W0 * m->D[r] + sum_t) / W1;
        m->W[r] = W1;

        if (last) {
            /* the most recent measurement: pairs of a voxel are in point
             * order, and a ray visits a voxel at most once */
            int64_t j = ord[e - 1].pid;
            double *st = m->sem + r * nsem;
            if (m->sem_mode == OM_SEM_CLOSED_LAST) st[0] = (double)last_class(m, sem, kind, j);
            else sem_row(m, sem, kind, j, st);
        } else if (rowlen) {
            if (n > rowcap) {
                free(rows);
                rowcap = n;
                rows = (double *)malloc((size_t)rowcap * (size_t)rowlen * sizeof(double));
                if (!rows) { free(ord); return -1; }
            }
            for (int64_t i = s; i < e; ++i) sem_row(m, sem, kind, ord[i].pid, rows + (i - s) * rowlen);
            double *st = m->sem + r * nsem;
            if (m->sem_mode == OM_SEM_CLOSED) {
                /* Eq. (6): concentrations grow by the (expected) class counts */
                for (int k = 0; k < rowlen; ++k) {
                    double c = 0.0;
                    for (int64_t i = 0; i < n; ++i) c += rows[i * rowlen + k];
                    st[k] += c;
                }
            } else {
                /* Eqs. (11)-(14) with lambda = W (previous), 2 nu = W, a batch
                 * of n observations with mean zbar. m at st[0..L), beta at
                 * st[L..2L). */
                double *mm = st, *bb = st + rowlen;
                for (int d = 0; d < rowlen; ++d) {
                    double z = 0.0;
                    for (int64_t i = 0; i < n; ++i) z += rows[i * rowlen + d];
                    double zbar = z / (double)n;
                    double ss = 0.0;
                    for (int64_t i = 0; i < n; ++i) {
                        double dz = rows[i * rowlen + d] - zbar;
                        ss += dz * dz;
                    }
                    double dm = zbar - mm[d];
                    bb[d] = bb[d] + 0.5 * ss + (W0 * (double)n / W1) * dm * dm / 2.0;
                    mm[d] = (W0 * mm[d] + (double)n * zbar) / W1;
                }
            }
        }
        s = e;
    }
    free(ord);
    free(rows);
    return 0;
}

/* Integrates one frame: pairs, then one batch (mode 0) or sequential (mode 1)
 * application.  Returns 0, or -1 on allocation failure. */
int om_integrate(omap *m, const float *pts, int64_t n, const double pose[16], const void *sem, int kind, int mode)
{
    m->st_points = n;
    m->st_rejected = 0;
    m->st_pairs = 0;
    m->st_uold = 0;
    m->st_unew = 0;
    m->st_newleaf = 0;
    int64_t rej = 0;
    int64_t P = om_frame_pairs(m, pts, n, pose, sem, kind, NULL, NULL, NULL, NULL, 0, &rej);
    int32_t *keys = (int32_t *)malloc((size_t)(P > 0 ? P : 1) * 3 * sizeof(int32_t));
    uint32_t *pid = (uint32_t *)malloc((size_t)(P > 0 ? P : 1) * sizeof(uint32_t));
    double *ts = (double *)malloc((size_t)(P > 0 ? P : 1) * sizeof(double));
    float *s32 = (float *)malloc((size_t)(P > 0 ? P : 1) * sizeof(float));
    if (!keys || !pid || !ts || !s32) { free(keys); free(pid); free(ts); free(s32); return -1; }
    om_frame_pairs(m, pts, n, pose, sem, kind, keys, pid, ts, s32, P, &rej);
    m->st_rejected = rej;
    m->st_pairs = P;
    int rc = om_apply(m, P, keys, pid, ts, sem, kind, mode);
    free(keys); free(pid); free(ts); free(s32);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* read-out                                                                  */
/* ------------------------------------------------------------------------- */

int64_t om_count(const omap *m) { return m->nvox; }
int64_t om_leaf_count(const omap *m) { return m->nleaf; }

/* points, rejected, pairs, voxels touched that existed, voxels created,
 * leaves created (last frame); total voxels; total leaves */
void om_stats(const omap *m, int64_t out[8])
{
    out[0] = m->st_points; out[1] = m->st_rejected; out[2] = m->st_pairs;
    out[3] = m->st_uold; out[4] = m->st_unew; out[5] = m->st_newleaf;
    out[6] = m->nvox; out[7] = m->nleaf;
}

typedef struct { int32_t lk[3], off[3]; int64_t r; } oext;

static int cmp_ext(const void *a, const void *b)
{
    const oext *x = (const oext *)a, *y = (const oext *)b;
    for (int i = 0; i < 3; ++i) if (x->lk[i] != y->lk[i]) return x->lk[i] < y->lk[i] ? -1 : 1;
    for (int i = 0; i < 3; ++i) if (x->off[i] != y->off[i]) return x->off[i] < y->off[i] ? -1 : 1;
    return 0;
}

/* Writes every voxel with W > 0, ordered by its 8^3 leaf (x, then y, then z
 * of the leaf coordinate) and then by its position inside the leaf (x, y, z).
 * keys: M x 3; D, W: M; sem: M x nsem (class counts; m then beta; the class
 * index (closed last); the embedding (open last)).
 * Returns M; writes nothing if cap < M. */
int64_t om_extract(const omap *m, int32_t *keys, double *D, double *W, double *sem, int64_t cap)
{
    if (cap < m->nvox) return m->nvox;
    oext *e = (oext *)malloc((size_t)(m->nvox > 0 ? m->nvox : 1) * sizeof(oext));
    for (int64_t r = 0; r < m->nvox; ++r) {
        int32_t c[3];
        unpack3(m->vkey[r], c);
        for (int a = 0; a < 3; ++a) {
            e[r].lk[a] = floor_div8(c[a]);
            e[r].off[a] = c[a] - 8 * e[r].lk[a];
        }
        e[r].r = r;
    }
    qsort(e, (size_t)m->nvox, sizeof(oext), cmp_ext);
    for (int64_t i = 0; i < m->nvox; ++i) {
        int64_t r = e[i].r;
        for (int a = 0; a < 3; ++a) keys[3 * i + a] = 8 * e[i].lk[a] + e[i].off[a];
        D[i] = m->D[r];
        W[i] = m->W[r];
        if (m->nsem) memcpy(sem + i * m->nsem, m->sem + r * m->nsem, (size_t)m->nsem * sizeof(double));
    }
    free(e);
    return m->nvox;
}

/* ------------------------------------------------------------------------- */
/* render: the map seen from a camera (the role NanoVDB plays in Sec. III-E) */
/* ------------------------------------------------------------------------- */

/* Casts one ray per pixel of a pinhole camera (pose map_T_camera, FP64;
 * intrinsics fx, fy, cx, cy) through the map and finds the first surface: the
 * first two consecutive cells of the Amanatides-Woo walk over [near, far] that
 * are both observed with D > 0 in front and D <= 0 behind.  The pixel direction
 * is ((u - cx) / fx, (v - cy) / fy, 1) in binary32, turned into the unit map
 * direction exactly as a sensor point is (same operations); the walk is the
 * integration walk with at most 3 ceil((far - near) / vs) + 4 cells and stops
 * at a cell outside the key range.  Outputs per pixel i = v * width + u:
 * depth[i], the distance along the ray where D, interpolated linearly between
 * the two cell centres' projections onto the ray, crosses zero (NaN: no
 * surface); key[3 i ..], the cell behind the surface (the first with D <= 0);
 * label[i], that cell's class (closed set: first largest count; most-recent
 * closed set: the stored class; else -1; -1 without a surface); margin[i], the
 * smallest |D| over the observed cells the walk met up to the surface (or over
 * the whole walk), which tells how close the sign decisions came to a tie. */
void om_render(const omap *m, const double pose[16], float fx, float fy, float cx, float cy, int width, int height,
               float near_t, float far_t, double *depth, int32_t *key, int32_t *label, double *margin)
{
    oframe f;
    frame_setup(m, pose, &f);
    int maxsteps = 3 * (int)ceil(((double)far_t - (double)near_t) / (double)m->vs) + 4;
    int32_t(*cells)[3] = (int32_t(*)[3])malloc((size_t)maxsteps * sizeof(*cells));
    for (int v = 0; v < height; ++v)
        for (int uu = 0; uu < width; ++uu) {
            int64_t i = (int64_t)v * width + uu;
            depth[i] = NAN;
            key[3 * i] = key[3 * i + 1] = key[3 * i + 2] = 0;
            label[i] = -1;
            margin[i] = INFINITY;
            float dc[3] = {((float)uu - cx) / fx, ((float)v - cy) / fy, 1.0f};
            float p[3], d[3], u[3];
            for (int a = 0; a < 3; ++a)
                p[a] = fmaf(f.R[a * 3 + 0], dc[0], fmaf(f.R[a * 3 + 1], dc[1], fmaf(f.R[a * 3 + 2], dc[2], f.t[a])));
            for (int a = 0; a < 3; ++a) d[a] = p[a] - f.t[a];
            float r = sqrtf(fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0])));
            if (!(r > 0.0f) || !isfinite(r)) continue;
            for (int a = 0; a < 3; ++a) u[a] = d[a] / r;
            int nv = band_walk(m->vs, maxsteps, f.t, u, near_t, far_t, cells);
            int have_prev = 0;
            double Dp = 0.0, sp = 0.0;
            for (int k = 0; k < nv; ++k) {
                int64_t ka[3];
                int inrange = 1;
                for (int a = 0; a < 3; ++a) {
                    ka[a] = (int64_t)f.a[a] + cells[k][a];
                    if (!(ka[a] > -OM_KEY_LIMIT && ka[a] < OM_KEY_LIMIT)) inrange = 0;
                }
                if (!inrange) break;
                int64_t pos = table_find(m->hkey, m->hcap, pack3((int32_t)ka[0], (int32_t)ka[1], (int32_t)ka[2]));
                if (pos < 0) {
                    have_prev = 0;
                    continue;
                }
                int64_t rec = m->hval[pos];
                double D = m->D[rec];
                if (fabs(D) < margin[i]) margin[i] = fabs(D);
                double sk = 0.0;
                for (int a = 0; a < 3; ++a)
                    sk += (((double)cells[k][a] + 0.5) * (double)m->vs - (double)f.t[a]) * (double)u[a];
                if (have_prev && Dp > 0.0 && D <= 0.0) {
                    depth[i] = sp + (sk - sp) * Dp / (Dp - D);
                    for (int a = 0; a < 3; ++a) key[3 * i + a] = (int32_t)ka[a];
                    if (m->sem_mode == OM_SEM_CLOSED) {
                        const double *c = m->sem + rec * m->nsem;
                        int best = 0;
                        for (int q = 1; q < m->K; ++q)
                            if (c[q] > c[best]) best = q;
                        label[i] = best;
                    } else if (m->sem_mode == OM_SEM_CLOSED_LAST) {
                        label[i] = (int32_t)m->sem[rec];
                    }
                    break;
                }
                have_prev = 1;
                Dp = D;
                sp = sk;
            }
        }
    free(cells);
}
