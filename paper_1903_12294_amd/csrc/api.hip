// Host side of the C ABI (include/mf4d.h): validation, device buffers, stream
// ordering and the round loop of the grower.
#include <mf4d.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "mf4d_internal.h"

using namespace mf4d;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(e_ == hipErrorOutOfMemory ? MF4D_ERR_OOM : MF4D_ERR_HIP,        \
                        "%s failed: %s", #expr, hipGetErrorString(e_));                 \
    } while (0)

template <class T>
int dev_alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? MF4D_ERR_OOM : MF4D_ERR_HIP,
                    "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    return MF4D_OK;
}

template <class T>
void dev_free(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return ((1 << r) == v) ? r : -1;
}

}  // namespace

struct mf4d_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int bt = 8;

    bool has_field = false;
    Geom g{};
    float* field = nullptr;
    uint32_t* Af = nullptr;
    uint32_t* Lf = nullptr;
    uint8_t* active = nullptr;
    uint8_t* dirty = nullptr;
    uint32_t* work = nullptr;

    bool has_particles = false;
    PGeom pg{};
    uint32_t* bins = nullptr;
    float* attr_t = nullptr;
    unsigned long long* Ap = nullptr;
    unsigned long long* Lp = nullptr;
    uint2* pend[2] = {nullptr, nullptr};
    uint32_t* pdirty = nullptr;
    uint32_t* dlist = nullptr;

    uint32_t* counters = nullptr;
    unsigned long long* stat64 = nullptr;
    uint32_t* h_counters = nullptr;
    unsigned long long* h_stat = nullptr;

    bool has_crit = false;
    float crit[4] = {0, 0, 0, 0};
    int32_t* seeds = nullptr;
    int64_t S = 0;
    int64_t seeds_cap = 0;
    int64_t max_rounds = 0;

    // grow state: 0 nothing grown, 1 converged, 2 stopped by the round cap
    int state = 0;
    int cur = 0;
    uint32_t last_npend = 0;
    mf4d_stats stats{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};

    void* staging = nullptr;
    size_t staging_bytes = 0;
};

namespace {

void free_field(mf4d_ctx* c) {
    dev_free(c->field);
    dev_free(c->Af);
    dev_free(c->Lf);
    dev_free(c->active);
    dev_free(c->dirty);
    dev_free(c->work);
    c->has_field = false;
}

void free_particles(mf4d_ctx* c) {
    dev_free(c->bins);
    dev_free(c->attr_t);
    dev_free(c->Ap);
    dev_free(c->Lp);
    dev_free(c->pend[0]);
    dev_free(c->pend[1]);
    dev_free(c->pdirty);
    dev_free(c->dlist);
    c->has_particles = false;
    c->pg = PGeom{};
}

int staging_for(mf4d_ctx* c, size_t bytes, void** out) {
    if (c->staging_bytes < bytes) {
        if (c->staging) (void)hipFree(c->staging);
        c->staging = nullptr;
        c->staging_bytes = 0;
        int rc = dev_alloc((char**)&c->staging, bytes);
        if (rc) return rc;
        c->staging_bytes = bytes;
    }
    *out = c->staging;
    return MF4D_OK;
}

int sync(mf4d_ctx* c) {
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MF4D_OK;
}

int read_counters(mf4d_ctx* c) {
    HIP_TRY(hipMemcpyAsync(c->h_counters, c->counters, C_NCOUNTERS * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

// The round loop: compact the dirty tiles into a work list; stop when it is
// empty; else sweep those tiles, then pull particle-steps whose voxel joined,
// close the trajectories of particles that gained steps and push their voxels.
int run_rounds(mf4d_ctx* c, int64_t* rounds_done) {
    int64_t r = 0;
    const bool parts = c->has_particles;
    while (true) {
        launch_fill_u32(c->counters + C_NWORK, 0, 1, c->stream);
        launch_compact_tiles(c->g, c->dirty, c->work, c->counters + C_NWORK, c->stream);
        int rc = read_counters(c);
        if (rc) return rc;
        const uint32_t nwork = c->h_counters[C_NWORK];
        if (nwork == 0) {
            c->state = 1;
            break;
        }
        if (c->max_rounds > 0 && r >= c->max_rounds) {
            // keep the work list for a resume: its tiles go back to dirty
            launch_mark_work(c->work, c->counters + C_NWORK, nwork, c->dirty, c->stream);
            c->state = 2;
            break;
        }
        launch_sweep(c->g, c->Af, c->Lf, c->active, c->work, c->counters + C_NWORK, nwork, c->dirty,
                     c->stat64 + S_TILE_VISITS, c->stream);
        if (parts) {
            const int nx = 1 - c->cur;
            const uint32_t npend = c->h_counters[C_PEND0 + c->cur];
            launch_fill_u32(c->counters + C_PEND0 + nx, 0, 1, c->stream);
            launch_fill_u32(c->counters + C_NDIRTYP, 0, 1, c->stream);
            launch_pull(c->pg, c->pend[c->cur], c->counters + C_PEND0 + c->cur, npend, c->pend[nx],
                        c->counters + C_PEND0 + nx, c->Lf, c->Lp, c->pdirty, c->dlist,
                        c->counters + C_NDIRTYP, c->stream);
            launch_close_push(c->g, c->pg, c->dlist, c->counters + C_NDIRTYP,
                              (uint32_t)(c->pg.P < (1 << 20) ? c->pg.P : (1 << 20)), c->Ap, c->Lp,
                              c->pdirty, c->bins, c->Af, c->Lf, c->active, c->dirty,
                              c->stat64 + S_PART_VISITS, c->stream);
            c->cur = nx;
        }
        ++r;
    }
    *rounds_done = r;
    return MF4D_OK;
}

int finish_stats(mf4d_ctx* c, mf4d_stats* out, bool fresh, int64_t rounds) {
    HIP_TRY(hipMemcpyAsync(c->h_stat, c->stat64, S_NSTAT * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_counters, c->counters, C_NCOUNTERS * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, c->stream));
    int rc = sync(c);
    if (rc) return rc;
    mf4d_stats& s = c->stats;
    if (fresh) s = mf4d_stats{};
    s.rounds += rounds;
    s.tile_visits = (int64_t)c->h_stat[S_TILE_VISITS];
    s.particle_visits = (int64_t)c->h_stat[S_PART_VISITS];
    s.active_tiles = (int64_t)c->h_stat[S_ACTIVE_TILES];
    s.seeds_dropped = (int64_t)c->h_counters[C_DROPPED];
    s.members_field = -1;
    s.members_particle = c->has_particles ? -1 : 0;
    float ms = 0;
    if (fresh) {
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        s.ms_admit_field = ms;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[2]));
        s.ms_admit = ms;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
        s.ms_rounds = ms;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[3]));
        s.ms_total = ms;
    } else {
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
        s.ms_rounds += ms;
        s.ms_total += ms;
    }
    if (out) *out = s;
    return MF4D_OK;
}

}  // namespace

extern "C" {

const char* mf4d_version(void) { return "mf4d 0.1.0 (gfx950)"; }

const char* mf4d_last_error(void) { return g_err.c_str(); }

int mf4d_create(mf4d_ctx** out, int device, void* hip_stream) {
    if (!out) return fail(MF4D_ERR_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(MF4D_ERR_ARG, "device %d of %d", device, n);
    HIP_TRY(hipSetDevice(device));
    mf4d_ctx* c = new (std::nothrow) mf4d_ctx();
    if (!c) return fail(MF4D_ERR_OOM, "host allocation failed");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    int rc = dev_alloc(&c->counters, C_NCOUNTERS);
    if (!rc) rc = dev_alloc(&c->stat64, S_NSTAT);
    if (!rc && hipHostMalloc((void**)&c->h_counters, C_NCOUNTERS * sizeof(uint32_t)) != hipSuccess)
        rc = fail(MF4D_ERR_OOM, "pinned host allocation failed");
    if (!rc && hipHostMalloc((void**)&c->h_stat, S_NSTAT * sizeof(unsigned long long)) != hipSuccess)
        rc = fail(MF4D_ERR_OOM, "pinned host allocation failed");
    for (int i = 0; !rc && i < 4; ++i)
        if (hipEventCreate(&c->ev[i]) != hipSuccess) rc = fail(MF4D_ERR_HIP, "hipEventCreate failed");
    if (rc) {
        mf4d_destroy(c);
        return rc;
    }
    *out = c;
    return MF4D_OK;
}

void mf4d_destroy(mf4d_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_field(c);
    free_particles(c);
    dev_free(c->counters);
    dev_free(c->stat64);
    dev_free(c->seeds);
    if (c->staging) (void)hipFree(c->staging);
    if (c->h_counters) (void)hipHostFree(c->h_counters);
    if (c->h_stat) (void)hipHostFree(c->h_stat);
    for (int i = 0; i < 4; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    delete c;
}

int mf4d_set_tile(mf4d_ctx* c, int bt) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (bt != 4 && bt != 8 && bt != 16) return fail(MF4D_ERR_ARG, "tile t-extent %d not in {4,8,16}", bt);
    if (c->has_field) return fail(MF4D_ERR_STATE, "tile shape must be set before the field is loaded");
    c->bt = bt;
    return MF4D_OK;
}

int mf4d_load_field(mf4d_ctx* c, const float* field, int X, int Y, int Z, int T, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!field) return fail(MF4D_ERR_ARG, "field is NULL");
    if (X <= 0 || Y <= 0 || Z <= 0 || T <= 0) return fail(MF4D_ERR_ARG, "dims must be positive");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    Geom g{};
    g.X = X; g.Y = Y; g.Z = Z; g.T = T;
    g.BT = c->bt;
    g.logBT = ilog2(c->bt);
    g.NXt = (X + 31) / 32;
    g.NYt = (Y + 7) / 8;
    g.NZt = (Z + 7) / 8;
    g.NTt = (T + g.BT - 1) / g.BT;
    const uint64_t nt = (uint64_t)g.NXt * g.NYt * g.NZt * g.NTt;
    g.WPT = 64u * g.BT;
    g.nwords = nt * g.WPT;
    if (g.nwords * 32ull >= (1ull << 32) || (uint64_t)X * Y * Z * T >= (1ull << 32) - 1)
        return fail(MF4D_ERR_UNSUPPORTED, "grid of %llu voxel-steps (padded %llu) needs >= 2^32 bits",
                    (unsigned long long)X * Y * Z * T, (unsigned long long)g.nwords * 32ull);
    g.NT = (uint32_t)nt;
    HIP_TRY(hipSetDevice(c->device));
    free_particles(c);
    free_field(c);
    c->state = 0;
    const size_t V = (size_t)X * Y * Z * T;
    int rc = dev_alloc(&c->field, V);
    if (!rc) rc = dev_alloc(&c->Af, g.nwords);
    if (!rc) rc = dev_alloc(&c->Lf, g.nwords);
    if (!rc) rc = dev_alloc(&c->active, (size_t)g.NT + 4);
    if (!rc) rc = dev_alloc(&c->dirty, (size_t)g.NT + 4);
    if (!rc) rc = dev_alloc(&c->work, g.NT);
    if (rc) {
        free_field(c);
        return rc;
    }
    HIP_TRY(hipMemcpyAsync(c->field, field, V * sizeof(float),
                           where == MF4D_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                           c->stream));
    launch_fill_u32(c->Af, 0, g.nwords, c->stream);
    launch_fill_u32(c->Lf, 0, g.nwords, c->stream);
    rc = sync(c);
    if (rc) {
        free_field(c);
        return rc;
    }
    c->g = g;
    c->has_field = true;
    return MF4D_OK;
}

int mf4d_load_particles(mf4d_ctx* c, const float* xyz, const float* attr, int64_t P, int T,
                        int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->has_field) return fail(MF4D_ERR_STATE, "load the field before the particles");
    if (P < 0) return fail(MF4D_ERR_ARG, "P < 0");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    if (P > 0 && (!xyz || !attr)) return fail(MF4D_ERR_ARG, "xyz or attr is NULL");
    if (P > 0 && T != c->g.T) return fail(MF4D_ERR_ARG, "particle T %d differs from field T %d", T, c->g.T);
    PGeom pg{};
    pg.P = P;
    pg.T = c->g.T;
    if (pg.T <= 64) {
        int tp = 1;
        while (tp < pg.T) tp <<= 1;
        pg.Tpad = tp;
    } else {
        pg.Tpad = (pg.T + 63) / 64 * 64;
    }
    pg.W = pg.Tpad <= 64 ? 1 : pg.Tpad / 64;
    pg.logTpad = ilog2(pg.Tpad);
    if ((uint64_t)P * pg.Tpad >= (1ull << 31))
        return fail(MF4D_ERR_UNSUPPORTED, "%lld particles x %d padded steps exceed 2^31",
                    (long long)P, pg.Tpad);
    HIP_TRY(hipSetDevice(c->device));
    free_particles(c);
    c->state = 0;
    if (P == 0) return MF4D_OK;
    const size_t Q = (size_t)P * pg.Tpad;
    int rc = dev_alloc(&c->bins, Q);
    if (!rc) rc = dev_alloc(&c->attr_t, Q);
    if (!rc) rc = dev_alloc(&c->Ap, (size_t)P * pg.W);
    if (!rc) rc = dev_alloc(&c->Lp, (size_t)P * pg.W);
    if (!rc) rc = dev_alloc(&c->pend[0], Q);
    if (!rc) rc = dev_alloc(&c->pend[1], Q);
    if (!rc) rc = dev_alloc(&c->pdirty, (size_t)(P + 31) / 32);
    if (!rc) rc = dev_alloc(&c->dlist, (size_t)P);
    if (rc) {
        free_particles(c);
        return rc;
    }
    const float* dx = xyz;
    const float* da = attr;
    float* tmp = nullptr;
    const size_t nxyz = (size_t)P * pg.T * 3, nat = (size_t)P * pg.T;
    if (where == MF4D_HOST) {
        rc = dev_alloc(&tmp, nxyz + nat);
        if (rc) {
            free_particles(c);
            return rc;
        }
        hipError_t e = hipMemcpyAsync(tmp, xyz, nxyz * sizeof(float), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(tmp + nxyz, attr, nat * sizeof(float), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            free_particles(c);
            return fail(MF4D_ERR_HIP, "particle upload failed: %s", hipGetErrorString(e));
        }
        dx = tmp;
        da = tmp + nxyz;
    }
    launch_bin_particles(c->g, pg, dx, da, c->bins, c->attr_t, c->stream);
    launch_fill_u32(c->pdirty, 0, (P + 31) / 32, c->stream);
    rc = sync(c);
    if (tmp) (void)hipFree(tmp);
    if (rc) {
        free_particles(c);
        return rc;
    }
    c->pg = pg;
    c->has_particles = true;
    return MF4D_OK;
}

int mf4d_set_criteria(mf4d_ctx* c, float f_lo, float f_hi, float a_lo, float a_hi) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (f_lo != f_lo || f_hi != f_hi || a_lo != a_lo || a_hi != a_hi)
        return fail(MF4D_ERR_ARG, "a criterion bound is NaN");
    c->crit[0] = f_lo;
    c->crit[1] = f_hi;
    c->crit[2] = a_lo;
    c->crit[3] = a_hi;
    c->has_crit = true;
    c->state = 0;
    return MF4D_OK;
}

int mf4d_set_seeds(mf4d_ctx* c, const int32_t* xyzt, int64_t S, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->has_field) return fail(MF4D_ERR_STATE, "load the field before the seeds");
    if (S < 0 || (S > 0 && !xyzt)) return fail(MF4D_ERR_ARG, "bad seed array");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    if (S > (1ll << 30)) return fail(MF4D_ERR_UNSUPPORTED, "too many seeds");
    HIP_TRY(hipSetDevice(c->device));
    // validate on the host (device seeds are copied down for this)
    int32_t* h = nullptr;
    const int32_t* hv = xyzt;
    if (S > 0 && where == MF4D_DEVICE) {
        h = new (std::nothrow) int32_t[S * 4];
        if (!h) return fail(MF4D_ERR_OOM, "host allocation failed");
        hipError_t e = hipMemcpy(h, xyzt, S * 4 * sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            delete[] h;
            return fail(MF4D_ERR_HIP, "seed download failed: %s", hipGetErrorString(e));
        }
        hv = h;
    }
    for (int64_t i = 0; i < S; ++i) {
        const int32_t* s = hv + 4 * i;
        if (s[0] < 0 || s[0] >= c->g.X || s[1] < 0 || s[1] >= c->g.Y || s[2] < 0 ||
            s[2] >= c->g.Z || s[3] < 0 || s[3] >= c->g.T) {
            delete[] h;
            return fail(MF4D_ERR_RANGE, "seed %lld (%d,%d,%d,%d) outside the %dx%dx%dx%d grid",
                        (long long)i, s[0], s[1], s[2], s[3], c->g.X, c->g.Y, c->g.Z, c->g.T);
        }
    }
    if (S > c->seeds_cap) {
        int32_t* ns = nullptr;
        int rc = dev_alloc(&ns, (size_t)S * 4);
        if (rc) {
            delete[] h;
            return rc;
        }
        dev_free(c->seeds);
        c->seeds = ns;
        c->seeds_cap = S;
    }
    if (S > 0) {
        hipError_t e = hipMemcpyAsync(c->seeds, hv, S * 4 * sizeof(int32_t),
                                      where == MF4D_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                      c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        delete[] h;
        if (e != hipSuccess) return fail(MF4D_ERR_HIP, "seed upload failed: %s", hipGetErrorString(e));
    }
    c->S = S;
    c->state = 0;
    return MF4D_OK;
}

int mf4d_set_max_rounds(mf4d_ctx* c, int64_t cap) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (cap < 0) return fail(MF4D_ERR_ARG, "cap < 0");
    c->max_rounds = cap;
    return MF4D_OK;
}

int mf4d_grow(mf4d_ctx* c, mf4d_stats* out) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->has_field) return fail(MF4D_ERR_STATE, "no field loaded");
    if (!c->has_crit) return fail(MF4D_ERR_STATE, "no criteria set");
    HIP_TRY(hipSetDevice(c->device));
    const Geom& g = c->g;
    hipStream_t s = c->stream;
    c->state = 0;
    launch_fill_u32(c->Lf, 0, g.nwords, s);
    launch_fill_u32((uint32_t*)c->active, 0, (g.NT + 3) / 4, s);
    launch_fill_u32((uint32_t*)c->dirty, 0, (g.NT + 3) / 4, s);
    launch_fill_u32(c->counters, 0, C_NCOUNTERS, s);
    launch_fill_u32((uint32_t*)c->stat64, 0, S_NSTAT * 2, s);
    if (c->has_particles) {
        launch_fill_u32((uint32_t*)c->Lp, 0, (uint64_t)c->pg.P * c->pg.W * 2, s);
        launch_fill_u32(c->pdirty, 0, (uint64_t)(c->pg.P + 31) / 32, s);
    }
    HIP_TRY(hipEventRecord(c->ev[0], s));
    launch_admit_field(g, c->field, c->crit[0], c->crit[1], c->Af, c->active, s);
    HIP_TRY(hipEventRecord(c->ev[1], s));
    if (c->has_particles)
        launch_admit_particles(c->pg, c->attr_t, c->bins, c->crit[2], c->crit[3], c->Ap, c->pend[0],
                               c->counters + C_PEND0, s);
    HIP_TRY(hipEventRecord(c->ev[2], s));
    launch_count_active(g, c->active, c->stat64 + S_ACTIVE_TILES, s);
    launch_seeds(g, c->seeds, c->S, c->Af, c->Lf, c->active, c->dirty, c->counters + C_DROPPED, s);
    c->cur = 0;
    int64_t rounds = 0;
    int rc = run_rounds(c, &rounds);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(c->ev[3], s));
    rc = finish_stats(c, out, true, rounds);
    if (rc) return rc;
    if (c->state == 2) return fail(MF4D_ERR_NOT_CONVERGED, "stopped after %lld rounds", (long long)rounds);
    return MF4D_OK;
}

int mf4d_grow_resume(mf4d_ctx* c, mf4d_stats* out) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (c->state != 2) return fail(MF4D_ERR_STATE, "nothing to resume");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipEventRecord(c->ev[2], c->stream));
    int rc = MF4D_OK;
    int64_t rounds = 0;
    rc = run_rounds(c, &rounds);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(c->ev[3], c->stream));
    rc = finish_stats(c, out, false, rounds);
    if (rc) return rc;
    if (c->state == 2) return fail(MF4D_ERR_NOT_CONVERGED, "stopped after %lld more rounds", (long long)rounds);
    return MF4D_OK;
}

int mf4d_read_field_mask(mf4d_ctx* c, uint32_t* dst, size_t nwords, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (c->state == 0) return fail(MF4D_ERR_STATE, "nothing grown");
    if (!dst) return fail(MF4D_ERR_ARG, "dst is NULL");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    const uint64_t V = (uint64_t)c->g.X * c->g.Y * c->g.Z * c->g.T;
    const size_t need = (size_t)((V + 31) / 32);
    if (nwords < need) return fail(MF4D_ERR_ARG, "dst holds %zu words, %zu needed", nwords, need);
    HIP_TRY(hipSetDevice(c->device));
    uint32_t* out = dst;
    if (where == MF4D_HOST) {
        void* st = nullptr;
        int rc = staging_for(c, need * sizeof(uint32_t), &st);
        if (rc) return rc;
        out = (uint32_t*)st;
    }
    launch_fill_u32((uint32_t*)(c->stat64 + S_MEMBERS_F), 0, 2, c->stream);
    launch_read_field(c->g, c->Lf, out, c->stat64 + S_MEMBERS_F, c->stream);
    if (where == MF4D_HOST)
        HIP_TRY(hipMemcpyAsync(dst, out, need * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_stat + S_MEMBERS_F, c->stat64 + S_MEMBERS_F,
                           sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    int rc = sync(c);
    if (rc) return rc;
    c->stats.members_field = (int64_t)c->h_stat[S_MEMBERS_F];
    return MF4D_OK;
}

int mf4d_read_particle_mask(mf4d_ctx* c, uint8_t* dst, size_t n, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (c->state == 0) return fail(MF4D_ERR_STATE, "nothing grown");
    if (!c->has_particles) return fail(MF4D_ERR_STATE, "no particles loaded");
    if (!dst) return fail(MF4D_ERR_ARG, "dst is NULL");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    const size_t need = (size_t)c->pg.P * c->pg.T;
    if (n < need) return fail(MF4D_ERR_ARG, "dst holds %zu bytes, %zu needed", n, need);
    HIP_TRY(hipSetDevice(c->device));
    uint8_t* out = dst;
    if (where == MF4D_HOST) {
        void* st = nullptr;
        int rc = staging_for(c, need, &st);
        if (rc) return rc;
        out = (uint8_t*)st;
    }
    launch_fill_u32((uint32_t*)(c->stat64 + S_MEMBERS_P), 0, 2, c->stream);
    launch_read_particles(c->pg, c->Lp, out, c->stat64 + S_MEMBERS_P, c->stream);
    if (where == MF4D_HOST)
        HIP_TRY(hipMemcpyAsync(dst, out, need, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_stat + S_MEMBERS_P, c->stat64 + S_MEMBERS_P,
                           sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    int rc = sync(c);
    if (rc) return rc;
    c->stats.members_particle = (int64_t)c->h_stat[S_MEMBERS_P];
    return MF4D_OK;
}

int mf4d_last_stats(mf4d_ctx* c, mf4d_stats* out) {
    if (!c || !out) return fail(MF4D_ERR_ARG, "NULL argument");
    if (c->state == 0) return fail(MF4D_ERR_STATE, "nothing grown");
    *out = c->stats;
    return MF4D_OK;
}

}  // extern "C"
