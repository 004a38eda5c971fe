// Host side of the C ABI (include/mf4d.h): validation, device buffers, stream
// ordering and the round loop of the grower.
#include <mf4d.h>

#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hipcub/hipcub.hpp>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

#include "mf4d_internal.h"
#include "batched.h"
#include "nn.h"
#include "slic.h"

#include <algorithm>
#include <vector>

using namespace mf4d;

namespace mf4d {
int net_infer(mf4d_net* n, const uint16_t* x, int N, int D, int H, int W, float* logits,
              hipStream_t s);
}

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

// Device memory held by the library's contexts, and an optional cap on it
// (MF4D_MAX_DEVICE_BYTES, read at each allocation): an allocation that would
// exceed the cap fails with MF4D_ERR_OOM as if the device were full, so that
// out-of-memory paths can be exercised on any GPU.
std::mutex g_mem_mu;
std::unordered_map<void*, size_t> g_mem_sizes;
size_t g_mem_total = 0;

size_t device_cap() {
    const char* e = getenv("MF4D_MAX_DEVICE_BYTES");
    if (!e || !*e) return SIZE_MAX;
    char* end = nullptr;
    const unsigned long long v = strtoull(e, &end, 10);
    return (end && *end == 0) ? (size_t)v : SIZE_MAX;
}

template <class T>
int dev_alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    std::lock_guard<std::mutex> lock(g_mem_mu);
    const size_t cap = device_cap();
    if (bytes > cap || g_mem_total > cap - bytes)
        return fail(MF4D_ERR_OOM, "allocation of %zu bytes exceeds MF4D_MAX_DEVICE_BYTES (%zu held)", bytes,
                    g_mem_total);
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? MF4D_ERR_OOM : MF4D_ERR_HIP,
                    "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    g_mem_sizes[(void*)*p] = bytes;
    g_mem_total += bytes;
    return MF4D_OK;
}

template <class T>
void dev_free(T*& p) {
    if (p) {
        (void)hipFree(p);
        std::lock_guard<std::mutex> lock(g_mem_mu);
        auto it = g_mem_sizes.find((void*)p);
        if (it != g_mem_sizes.end()) {
            g_mem_total -= it->second;
            g_mem_sizes.erase(it);
        }
    }
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
    int schedule = MF4D_SCHED_PERSISTENT;

    bool has_field = false;
    Geom g{};
    float* field = nullptr;
    uint32_t* Af = nullptr;
    uint32_t* Lf = nullptr;
    uint8_t* active = nullptr;
    uint32_t* dirty = nullptr;
    uint8_t* chg = nullptr;
    uint32_t* work = nullptr;
    float2* tsum = nullptr;
    uint32_t* cand = nullptr;
    int admit_all = 0;
    int forward_only = 0;  // trajectory coupling from t to t + 1 only

    bool has_particles = false;
    PGeom pg{};
    uint32_t* bins = nullptr;
    float* attr_t = nullptr;
    unsigned long long* Ap = nullptr;
    unsigned long long* Lp = nullptr;
    uint2* clist = nullptr;
    uint32_t* wcnt = nullptr;       // work sub-list lengths
    uint32_t* pdirty = nullptr;
    uint8_t* pflag = nullptr;       // P candidate flags
    uint32_t* dlist = nullptr;
    float2* psum = nullptr;

    // the statistics (S_NSTAT words) and right after them the counters
    // (C_NCOUNTERS), one allocation on the device and one on the host, so
    // that one copy brings both back
    uint32_t* counters = nullptr;
    unsigned long long* stat64 = nullptr;
    unsigned long long* slots = nullptr;  // per-block partial statistics
    uint32_t* bar = nullptr;
    uint32_t* h_counters = nullptr;
    unsigned long long* h_stat = nullptr;

    bool has_crit = false;
    float crit[4] = {0, 0, 0, 0};
    int32_t* seeds = nullptr;
    int64_t S = 0;
    int64_t seeds_cap = 0;
    int64_t max_rounds = 0;
    int64_t last_rounds = 0;  // rounds of the last grow that converged (launch mode)

    // grow state: 0 nothing grown, 1 converged, 2 stopped by the round cap
    int state = 0;
    uint32_t round = 0;  // index of the next round to run
    mf4d_stats stats{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t rev[4 * 4] = {};  // per launched round of a chunk: before sweep, pull, close, after
    double ms_phase[3] = {0, 0, 0};  // sweep, pull, close of the current grow
    bool members_pending[2] = {false, false};  // member counts in flight (field, particles)
    bool phase_timing = false;  // events around launched round kernels
    bool timed = false;         // the current grow records its events

    void* staging = nullptr;
    size_t staging_bytes = 0;

    // A second stream for the particle read-out, beside the field read-out
    // on the context stream; joined back into the context stream with an
    // event, so every call stays ordered on it.
    hipStream_t side = nullptr;
    hipEvent_t ev_labels = nullptr;   // recorded after the last work that changed the labels
    bool labels_marked = false;
    hipEvent_t ev_pread = nullptr;    // the particle read-out on the side stream is done
    bool stats_ready = false;         // h_stat / h_counters already hold this grow's statistics
    // read-outs of mf4d_grow_read, queued behind the rounds (device buffers)
    uint32_t* rd_f = nullptr;
    uint8_t* rd_p = nullptr;
    bool reads_done = false;          // the queued read-outs ran on the final labels
    hipEvent_t ev_chunk = nullptr;    // end of the last queued chunk of rounds
    hipEvent_t ev_stat = nullptr;     // its statistics copied to the host
    uint32_t* gsnap = nullptr;        // [2][C_NCOUNTERS]: chunk-end counters per label set (read gate)
    // Asynchronous read-outs (mf4d_set_read_async): a grow_read leaves its
    // read-outs deferred; the next asynchronous grow_read grows on the other
    // of two label sets and issues them on the side stream once its own
    // admissibility passes are queued, so they run beside its rounds; any
    // other call issues them at once.  The context stream waits for them
    // only when a later call needs it.  Set k's buffers are Lf / active / Lp
    // / pflag while it is current, the *_alt ones otherwise (swapped).
    bool read_async = false;
    bool async_grow = false;          // the grow in progress is an asynchronous grow_read
    struct {
        uint32_t* f;
        uint8_t* p;
        int set;
        bool valid;
    } dread = {nullptr, nullptr, 0, false};  // deferred read-outs of the last grow
    hipEvent_t ev_issue = nullptr;    // where deferred read-outs may start
    int issue_round = 1;              // launched rounds: issue them after this many rounds (measured:
                                      // after 0-2 alike, after 3 slower)
    int lset = 0;                     // index of the current label set
    uint32_t* Lf_alt = nullptr;
    uint8_t* active_alt = nullptr;
    unsigned long long* Lp_alt = nullptr;
    uint8_t* pflag_alt = nullptr;
    bool alt_ready = false;           // the other set's buffers hold no uninitialised words
    hipEvent_t ev_read[2] = {nullptr, nullptr};  // read-outs of label set k done
    bool read_pending[2] = {false, false};
    // A submitted grow (mf4d_grow_submit): 2 while its first chunk of rounds
    // and read-outs are queued and the host has not looked at them, 1 once
    // its result is kept for mf4d_grow_finish, 0 with none.
    int submitted = 0;
    Dev sub_d{};                      // its buffers and criteria
    int64_t sub_chunk = 0;            // rounds in its queued chunk
    int sub_npar = 0;
    uint32_t* sub_f = nullptr;
    size_t sub_nwords = 0;
    uint8_t* sub_p = nullptr;
    size_t sub_n = 0;
    int sub_rc = 0;
    std::string sub_err;
    mf4d_stats sub_stats{};

    // batched queries
    int Q = 0;
    float* btab = nullptr;
    int32_t* qseeds = nullptr;
    int64_t QS = 0, qseeds_cap = 0;
    uint32_t NTB = 0;
    int NXb = 0, NYb = 0, NZb = 0, NTb = 0;
    int blog[4] = {3, 2, 2, 2};  // log2 of the batched tile extents (x, y, z, t)
    uint8_t* b_active = nullptr;
    uint32_t* b_vrank = nullptr;  // [V] ranks of the voxel-steps under the query bands
    uint32_t* b_prank = nullptr;  // [P][Tpad] ranks of the particle-steps
    uint32_t* b_dirty = nullptr;
    uint8_t* b_chg = nullptr;
    uint32_t* b_work = nullptr;
    uint32_t* b_wcnt = nullptr;
    uint32_t b_wcap = 0;
    uint32_t* b_counters = nullptr;
    uint32_t* b_fown = nullptr;  // planes owned by the context (a batched grow given no buffers)
    uint32_t* b_pown = nullptr;
    size_t b_fown_n = 0, b_pown_n = 0;
    bool b_grown = false;        // the owned planes hold the last batched grow

    // brick statistics and the activity predictor
    BrickDims bd{};
    float4* bstats = nullptr;   // [T][Db][Hb][Wb] (min, max, mean, particle-steps)
    bool bstats_valid = false;  // computed on first use by the predictor
    uint16_t* feat = nullptr;   // bf16 [T][Db][Hb][Wb][16]
    float* blogits = nullptr;   // [T][Db][Hb][Wb]
    uint8_t* tpred = nullptr;   // NT
    mf4d_net* net = nullptr;
    mf4d_net* own_net = nullptr;  // the network of the learned scheduler (mf4d_set_scheduler)
    float pred_thr = 0.0f;
    // score-ordered schedulers (MF4D_SCHEDULER_LEARNED / _HEURISTIC): priority
    // list of the candidate tiles, sorted on the device
    int priority = MF4D_SCHEDULER_PLAIN;
    uint32_t* pr_buf = nullptr;  // 4 x NT: keys, tiles, sorted keys, sorted tiles; then the count
    void* pr_tmp = nullptr;      // radix sort scratch
    size_t pr_tmp_bytes = 0;
    int pr_waves = 512;          // wavefronts of the priority pass
    // Jacobi sweeps (MF4D_SCHED_JACOBI): the next labels
    uint32_t* jlf = nullptr;
    unsigned long long* jlp = nullptr;

    // particles as loaded, for the clustering: xyz [T][P][3] then attr [T][P]
    float* praw = nullptr;
    uint32_t* porder = nullptr;  // point samples sorted by tile (built on the first clustering)
    float4* spos = nullptr;      // their positions and times in that order
    float* sattr = nullptr;      // their values in that order
    // 4D SLIC clustering (Section 3.2)
    bool slic_params = false;
    int sk[4] = {1, 1, 1, 1};
    float swd = 1.0f, swf = 1.0f, swp = 1.0f, scf = 1.0f;
    double seps = 0.0;
    int smax_iter = 10;
    int sK = 0;
    int32_t* slabels = nullptr;  // [V + T * P]
    size_t slabels_n = 0;
    unsigned long long* sacc = nullptr;
    double* scen = nullptr;
    float* scen32 = nullptr;
    long long* scnt = nullptr;
    uint32_t* scounters = nullptr;
    uint32_t* h_scounters = nullptr;
    uint32_t* sslab = nullptr;  // 8 x 4096 slab bounds, then 8 x 4096 reach ranges (k_d <= 4096)
    unsigned long long* slsum = nullptr;  // [K][8] sums of the last update
    // cluster merging (Section 3.3), sized by K
    char* mbuf = nullptr;
    DevM m{};
    bool merged = false;
    bool slic_done = false;
    int slic_iters = 0;
};

namespace {

// Clustering labels (sized by the loaded samples); the centre buffers stay.
void free_slic(mf4d_ctx* c) {
    dev_free(c->slabels);
    c->slabels_n = 0;
    c->slic_done = false;
    c->merged = false;
}

void quiesce_side(mf4d_ctx* c) {
    if (c->side) (void)hipStreamSynchronize(c->side);
    c->labels_marked = false;
}

// Record that the labels are final up to here on the context stream: a
// read-out on the side stream waits for this event only.
void mark_labels(mf4d_ctx* c) {
    c->labels_marked = hipEventRecord(c->ev_labels, c->stream) == hipSuccess;
}

void free_field(mf4d_ctx* c) {
    quiesce_side(c);
    free_slic(c);
    dev_free(c->field);
    dev_free(c->Af);
    dev_free(c->Lf);
    dev_free(c->active);
    dev_free(c->Lf_alt);
    dev_free(c->active_alt);
    c->alt_ready = false;
    dev_free(c->dirty);
    dev_free(c->work);
    dev_free(c->wcnt);
    dev_free(c->chg);
    dev_free(c->tsum);
    dev_free(c->cand);
    dev_free(c->bstats);
    dev_free(c->feat);
    dev_free(c->blogits);
    dev_free(c->tpred);
    dev_free(c->pr_buf);
    dev_free(c->jlf);
    {
        char* tmp = static_cast<char*>(c->pr_tmp);
        dev_free(tmp);
        c->pr_tmp = nullptr;
        c->pr_tmp_bytes = 0;
    }
    dev_free(c->b_active);
    dev_free(c->b_vrank);
    dev_free(c->b_dirty);
    dev_free(c->b_chg);
    dev_free(c->b_work);
    dev_free(c->b_wcnt);
    dev_free(c->b_fown);
    dev_free(c->b_pown);
    c->b_fown_n = c->b_pown_n = 0;
    c->b_grown = false;
    c->NTB = 0;
    c->has_field = false;
}

void free_particles(mf4d_ctx* c) {
    quiesce_side(c);
    dev_free(c->jlp);
    dev_free(c->b_prank);
    dev_free(c->praw);
    dev_free(c->porder);
    dev_free(c->spos);
    dev_free(c->sattr);
    free_slic(c);
    dev_free(c->bins);
    dev_free(c->attr_t);
    dev_free(c->Ap);
    dev_free(c->Lp);
    dev_free(c->Lp_alt);
    dev_free(c->pflag_alt);
    c->alt_ready = false;
    dev_free(c->clist);
    dev_free(c->pdirty);
    dev_free(c->pflag);
    dev_free(c->dlist);
    dev_free(c->psum);
    dev_free(c->b_pown);
    c->b_pown_n = 0;
    c->b_grown = false;
    c->has_particles = false;
    c->pg = PGeom{};
    c->bstats_valid = false;
}

int staging_for(mf4d_ctx* c, size_t bytes, void** out) {
    if (c->staging_bytes < bytes) {
        char* old = static_cast<char*>(c->staging);
        dev_free(old);
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

constexpr size_t kStatBytes = S_NSTAT * sizeof(unsigned long long) + C_NCOUNTERS * sizeof(uint32_t);

int settle_submit(mf4d_ctx* c);

Dev make_dev(mf4d_ctx* c) {
    Dev d{};
    d.g = c->g;
    d.pg = c->pg;
    d.field = c->field;
    d.Af = c->Af;
    d.Lf = c->Lf;
    d.active = c->active;
    d.dirty = c->dirty;
    d.chg = c->chg;
    d.work = c->work;
    d.wcnt = c->wcnt;
    d.bins = c->bins;
    d.attr_t = c->attr_t;
    d.Ap = c->Ap;
    d.Lp = c->Lp;
    d.clist = c->clist;
    d.pdirty = c->pdirty;
    d.pflag = c->pflag;
    d.slots = c->slots;
    d.counters = c->counters;
    d.stat64 = c->stat64;
    d.bar = c->bar;
    d.tsum = c->tsum;
    d.psum = c->psum;
    d.cand = c->cand;
    d.tpred = nullptr;
    d.admit_all = c->admit_all || c->schedule == MF4D_SCHED_JACOBI;  // Jacobi sweeps read every word
    d.forward_only = c->forward_only;
    for (int i = 0; i < 4; ++i) d.crit[i] = c->crit[i];
    return d;
}

// The context's buffers with label set `set` (the current one or the other).
Dev make_dev_set(mf4d_ctx* c, int set) {
    Dev d = make_dev(c);
    if (set != c->lset) {
        d.Lf = c->Lf_alt;
        d.active = c->active_alt;
        d.Lp = c->Lp_alt;
        d.pflag = c->pflag_alt;
    }
    return d;
}

// Issue the deferred read-outs on the side stream after `after` (recorded on
// the context stream; null: now), from the label set they belong to.  last:
// they are the last grow's (its member counts are then the ones reported).
int issue_deferred(mf4d_ctx* c, hipEvent_t after, bool last) {
    if (!c->dread.valid) return MF4D_OK;
    c->dread.valid = false;
    if (!after) {
        HIP_TRY(hipEventRecord(c->ev_issue, c->stream));
        after = c->ev_issue;
    }
    HIP_TRY(hipStreamWaitEvent(c->side, after, 0));
    const Dev d = make_dev_set(c, c->dread.set);
    if (c->dread.p) {
        launch_read_particles(d, c->dread.p, c->side);
        launch_fold_slots(d, SL_MEMBERS_P, S_MEMBERS_P, c->side, true);
    }
    if (c->dread.f) {
        launch_read_field(d, c->dread.f, c->side);
        launch_fold_slots(d, SL_MEMBERS_F, S_MEMBERS_F, c->side, true);
    }
    HIP_TRY(hipEventRecord(c->ev_read[c->dread.set], c->side));
    c->read_pending[c->dread.set] = true;
    if (last) {
        c->members_pending[0] = c->dread.f != nullptr;
        c->members_pending[1] = c->dread.p != nullptr;
    }
    return MF4D_OK;
}

// Issue deferred read-outs and let the context stream wait for every
// asynchronous read-out still running: every call other than an
// asynchronous grow_read starts with it, so nothing it queues can touch
// labels, member counts or buffers those read-outs use.
int settle_async(mf4d_ctx* c) {
    settle_submit(c);
    int rc = issue_deferred(c, nullptr, true);
    if (rc) return rc;
    for (int k = 0; k < 2; ++k)
        if (c->read_pending[k]) {
            HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_read[k], 0));
            c->read_pending[k] = false;
        }
    return MF4D_OK;
}

// Queue the read-outs of mf4d_grow_read behind the rounds queued so far: the
// particle labels on the side stream after ev_chunk, the field labels on the
// context stream.  Gated on the chunk's counter copy: with a closed gate they
// do nothing.  The context stream's wait for the side stream is queued by the
// caller (join_reads).
int queue_reads(mf4d_ctx* c, const ReadGate& gate) {
    const Dev d = make_dev(c);
    hipStream_t s = c->stream;
    HIP_TRY(hipStreamWaitEvent(c->side, c->ev_chunk, 0));
    if (c->rd_p) {
        launch_read_particles(d, c->rd_p, c->side, gate);
        launch_fold_slots(d, SL_MEMBERS_P, S_MEMBERS_P, c->side, true);
    }
    if (c->rd_f) {
        launch_read_field(d, c->rd_f, s, gate);
        launch_fold_slots(d, SL_MEMBERS_F, S_MEMBERS_F, s, true);
    }
    HIP_TRY(hipEventRecord(c->ev_pread, c->side));
    return MF4D_OK;
}

// After a chunk's read-outs were queued: the context stream waits for the
// side stream's part.
int join_reads(mf4d_ctx* c) {
    if (!c->rd_p) return MF4D_OK;
    HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_pread, 0));
    return MF4D_OK;
}

// Statistics and counters to the host in one copy; read-outs pending are
// queued behind it (they run while the host waits for the copy only).
// queue_stat_copy queues; read_chunk also waits for the copy.
int queue_stat_copy(mf4d_ctx* c, const ReadGate& gate) {
    hipStream_t s = c->stream;
    HIP_TRY(hipEventRecord(c->ev_chunk, s));
    HIP_TRY(hipMemcpyAsync(c->h_stat, c->stat64, kStatBytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(c->ev_stat, s));
    if (c->rd_f || c->rd_p) {
        int rc = queue_reads(c, gate);
        if (rc) return rc;
    }
    HIP_TRY(hipGetLastError());
    return MF4D_OK;
}

// The host waits for a chunk's statistics by polling the event: a grow's
// rounds take well under a millisecond, and a blocking wait adds a wake-up to
// every grow while the device idles until the next grow is queued.
int wait_stat(mf4d_ctx* c) {
    hipError_t q;
    while ((q = hipEventQuery(c->ev_stat)) == hipErrorNotReady) {
    }
    HIP_TRY(q);
    return MF4D_OK;
}

int read_chunk(mf4d_ctx* c, const ReadGate& gate) {
    int rc = queue_stat_copy(c, gate);
    if (rc) return rc;
    return wait_stat(c);
}

// Jacobi sweeps until one adds nothing (converged) or the cap is hit; each
// sweep reads the current labels and writes a copy, then the copy becomes
// current.  rounds_done: the sweeps run (the last converged one included).
int run_jacobi(mf4d_ctx* c, const Dev& d, int64_t* rounds_done) {
    c->stats_ready = false;
    const uint64_t nw = c->g.nwords;
    const uint64_t np = c->has_particles ? (uint64_t)c->pg.P * c->pg.W : 0;
    int rc = MF4D_OK;
    if (!c->jlf) rc = dev_alloc(&c->jlf, nw);
    if (!rc && np && !c->jlp) rc = dev_alloc(&c->jlp, np);
    if (rc) return rc;
    hipStream_t s = c->stream;
    int64_t k = 0;
    while (true) {
        if (c->max_rounds > 0 && k >= c->max_rounds) {
            c->state = 2;
            break;
        }
        HIP_TRY(hipMemcpyAsync(c->jlf, c->Lf, nw * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        if (np) HIP_TRY(hipMemcpyAsync(c->jlp, c->Lp, np * sizeof(unsigned long long), hipMemcpyDeviceToDevice, s));
        launch_fill_u32(c->counters + C_JCHANGED, 0, 1, s);
        launch_jacobi(d, c->Lf, c->Lp, c->jlf, c->jlp, s);
        HIP_TRY(hipMemcpyAsync(c->Lf, c->jlf, nw * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        if (np) HIP_TRY(hipMemcpyAsync(c->Lp, c->jlp, np * sizeof(unsigned long long), hipMemcpyDeviceToDevice, s));
        rc = read_counters(c);
        if (rc) return rc;
        ++k;
        if (!c->h_counters[C_JCHANGED]) {
            c->state = 1;
            break;
        }
    }
    c->round += (uint32_t)k;
    *rounds_done = k;
    return MF4D_OK;
}

// Launched rounds are queued a chunk at a time (a round with an empty work
// list is a no-op on the device), and the host reads the counters once per
// chunk.  C_ROUNDS counts the rounds that had work.  Each host read costs
// about three queued empty rounds (measured), so the first chunk of a grow is
// as long as the context's last converged grow (4 to 16 rounds), the later
// ones kRoundChunk; with phase timing every chunk is kRoundChunk (one set of
// events per round).
struct RoundChunk {
    int64_t n;  // rounds queued (0: the round cap was reached)
    int npar;   // parity of the round after the chunk
};

// Queue the chunk of rounds that starts r rounds into the grow, its
// chunk-end kernel, the statistics copy and the read-outs pending (gated on
// this chunk reaching the fixed point).  The host does not wait.
int queue_chunk(mf4d_ctx* c, const Dev& d, int64_t r, RoundChunk* ch) {
    constexpr int64_t kRoundChunk = 4, kMaxChunk = 16;
    const uint32_t cap = (uint32_t)(c->max_rounds > 0 ? c->max_rounds : 0);
    int64_t chunk = kRoundChunk;
    if (r == 0 && !c->timed) chunk = std::min(std::max(c->last_rounds, kRoundChunk), kMaxChunk);
    if (cap && cap - r < chunk) chunk = cap - r;
    ch->n = chunk > 0 ? chunk : 0;
    ch->npar = 0;
    if (chunk <= 0) return MF4D_OK;
    for (int64_t k = 0; k < chunk; ++k) {
        launch_round(d, (uint32_t)(c->round + k), c->stream, c->timed ? c->rev + 4 * k : nullptr);
        if (c->async_grow && c->dread.valid && r == 0 && k + 1 == c->issue_round) {
            HIP_TRY(hipEventRecord(c->ev_issue, c->stream));
            int rc = issue_deferred(c, c->ev_issue, false);
            if (rc) return rc;
        }
    }
    // work total and the grow's statistics, read back together, so that
    // finish_stats needs no wait of its own after the last chunk
    const int npar = (int)((c->round + chunk) & 1);
    uint32_t* snap = (c->rd_f || c->rd_p) ? c->gsnap + c->lset * C_NCOUNTERS : nullptr;
    launch_chunk_end(d, npar, snap, c->stream);
    ch->npar = npar;
    return queue_stat_copy(c, ReadGate{snap, (uint32_t)(r + chunk), npar});
}

// Wait for a queued chunk's counters: the rounds it did (r advances by
// them) and whether the grow reached the fixed point.
int settle_chunk(mf4d_ctx* c, int64_t* r, const RoundChunk& ch, bool* converged) {
    int rc = wait_stat(c);
    if (rc) return rc;
    c->stats_ready = true;
    const int64_t done = (int64_t)c->h_counters[C_ROUNDS] - *r;
    for (int64_t k = 0; c->timed && k < done && k < ch.n; ++k)
        for (int ph = 0; ph < 3; ++ph) {
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, c->rev[4 * k + ph], c->rev[4 * k + ph + 1]));
            c->ms_phase[ph] += ms;
        }
    c->round += (uint32_t)done;
    *r += done;
    *converged = done < ch.n || c->h_counters[C_NWORK0 + (c->round & 1)] == 0;
    return join_reads(c);
}

// Rounds until a round's work list is empty (converged) or the cap is hit.
// Persistent: one cooperative launch runs every round; if it cannot be
// launched, or a grid barrier timed out, the rounds run as launches instead.
// queued: a first chunk of launched rounds already queued (a submitted grow).
int run_rounds(mf4d_ctx* c, const Dev& d, int64_t* rounds_done, const RoundChunk* queued = nullptr) {
    if (c->schedule == MF4D_SCHED_JACOBI) return run_jacobi(c, d, rounds_done);
    const uint32_t cap = (uint32_t)(c->max_rounds > 0 ? c->max_rounds : 0);
    const uint32_t r0 = c->round;
    if (c->schedule == MF4D_SCHED_PERSISTENT && !queued) {
        if (c->round != 0) {  // a fresh grow's reset cleared them
            launch_fill_u32(c->counters + C_ERR, 0, 2, c->stream);  // C_ERR, C_ROUNDS
            launch_fill_u32(c->bar, 0, kBarWords, c->stream);
        }
        if (launch_rounds_persistent(d, r0, cap, c->device, c->stream)) {
            launch_fold_grow_slots(d, c->stream);
            // read-outs pending run unconditionally: the launch ran every
            // round it was going to
            int rc = read_chunk(c, ReadGate{});
            if (rc) return rc;
            rc = join_reads(c);
            if (rc) return rc;
            c->reads_done = c->rd_f || c->rd_p;
            c->stats_ready = true;
            if (c->h_counters[C_ERR] == 0) {
                const uint32_t done = c->h_counters[C_ROUNDS];
                c->round = r0 + done;
                *rounds_done = done;
                c->state = c->h_counters[C_NWORK0 + (c->round & 1)] == 0 ? 1 : 2;
                return MF4D_OK;
            }
            return fail(MF4D_ERR_HIP, "persistent rounds: a grid barrier timed out");
        }
        (void)hipGetLastError();
    }
    // Launches: rounds are queued a chunk at a time (queue_chunk), the host
    // waiting for each chunk's counters (settle_chunk).
    if (!queued && c->round != 0) launch_fill_u32(c->counters + C_ROUNDS, 0, 1, c->stream);  // fresh: reset cleared it
    int64_t r = 0;
    RoundChunk ch{0, 0};
    if (queued) ch = *queued;
    while (true) {
        if (!queued) {
            int rc = queue_chunk(c, d, r, &ch);
            if (rc) return rc;
        }
        queued = nullptr;
        if (ch.n <= 0) {  // cap reached with work left
            c->state = 2;
            break;
        }
        bool converged = false;
        int rc = settle_chunk(c, &r, ch, &converged);
        if (rc) return rc;
        if (converged) {
            c->state = 1;
            c->reads_done = c->rd_f || c->rd_p;  // their gate was open
            break;
        }
    }
    *rounds_done = r;
    return MF4D_OK;
}

int finish_stats(mf4d_ctx* c, mf4d_stats* out, bool fresh, int64_t rounds) {
    if (!c->stats_ready) {  // else the last read of the rounds brought them
        launch_fold_grow_slots(make_dev(c), c->stream);
        HIP_TRY(hipMemcpyAsync(c->h_stat, c->stat64, kStatBytes, hipMemcpyDeviceToHost, c->stream));
        int rc = sync(c);
        if (rc) return rc;
    }
    c->stats_ready = false;
    // with phase timing the events after the last read must have completed
    if (c->timed) HIP_TRY(hipEventSynchronize(c->ev[3]));
    mf4d_stats& s = c->stats;
    if (fresh) s = mf4d_stats{};
    s.rounds += rounds;
    s.tile_visits = (int64_t)c->h_stat[S_TILE_VISITS];
    s.particle_visits = (int64_t)c->h_stat[S_PART_VISITS];
    s.active_tiles = (int64_t)c->h_stat[S_ACTIVE_TILES];
    if (fresh) s.tiles_tested = c->admit_all ? (int64_t)c->g.NT : (int64_t)c->h_stat[S_TILES_TESTED];
    s.tiles_deferred_read = (int64_t)c->h_stat[S_DEFERRED_READ];
    s.priority_visits = (int64_t)c->h_stat[S_PRIO_VISITS];
    s.ms_sweep = c->ms_phase[0];
    s.ms_pull = c->ms_phase[1];
    s.ms_close = c->ms_phase[2];
    if (fresh) s.coupled_steps = c->has_particles ? (int64_t)c->h_counters[C_NLIST] : 0;
    s.seeds_dropped = (int64_t)c->h_counters[C_DROPPED];
    s.members_field = -1;
    s.members_particle = c->has_particles ? -1 : 0;
    float ms = 0;
    if (!c->timed) {
        // no events were recorded: device times are reported only with phase timing on
    } else if (fresh) {
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

// Bumped whenever a kernel changes: autotuner caches and recorded hardware
// counter figures are keyed by it.
const char* mf4d_version(void) { return "mf4d 0.7.7 (gfx950)"; }

const char* mf4d_last_error(void) { return g_err.c_str(); }

int64_t mf4d_device_bytes(void) {
    std::lock_guard<std::mutex> lock(g_mem_mu);
    return (int64_t)g_mem_total;
}

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
    static_assert(C_NCOUNTERS % 2 == 0, "counters fill whole 8-byte words");
    int rc = dev_alloc(&c->stat64, S_NSTAT + C_NCOUNTERS / 2);
    if (!rc) c->counters = reinterpret_cast<uint32_t*>(c->stat64 + S_NSTAT);
    if (!rc) rc = dev_alloc(&c->bar, kBarWords);
    if (!rc) rc = dev_alloc(&c->gsnap, 2 * (size_t)C_NCOUNTERS);
    if (!rc) rc = dev_alloc(&c->slots, (size_t)kSlotStats * kSlots);
    if (!rc) launch_fill_u32((uint32_t*)c->slots, 0, 2ull * kSlotStats * kSlots, c->stream);
    if (!rc) {
        const char* env = getenv("MF4D_SCHED");
        if (env && strcmp(env, "launch") == 0) c->schedule = MF4D_SCHED_LAUNCH;
        const char* adm = getenv("MF4D_ADMIT");
        if (adm && strcmp(adm, "all") == 0) c->admit_all = 1;
    }
    if (!rc && hipHostMalloc((void**)&c->h_stat, kStatBytes) != hipSuccess)
        rc = fail(MF4D_ERR_OOM, "pinned host allocation failed");
    if (!rc) c->h_counters = reinterpret_cast<uint32_t*>(c->h_stat + S_NSTAT);
    for (int i = 0; !rc && i < 4; ++i)
        if (hipEventCreate(&c->ev[i]) != hipSuccess) rc = fail(MF4D_ERR_HIP, "hipEventCreate failed");
    for (int i = 0; !rc && i < 16; ++i)
        if (hipEventCreate(&c->rev[i]) != hipSuccess) rc = fail(MF4D_ERR_HIP, "hipEventCreate failed");
    if (!rc && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess)
        rc = fail(MF4D_ERR_HIP, "hipStreamCreateWithFlags failed");
    for (hipEvent_t* e : {&c->ev_labels, &c->ev_pread, &c->ev_chunk, &c->ev_stat, &c->ev_read[0], &c->ev_read[1], &c->ev_issue})
        if (!rc && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess)
            rc = fail(MF4D_ERR_HIP, "hipEventCreate failed");
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
    (void)settle_async(c);  // deferred read-outs still write the caller's buffers
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->side) (void)hipStreamSynchronize(c->side);
    free_field(c);
    free_particles(c);
    c->counters = nullptr;  // inside stat64
    dev_free(c->stat64);
    dev_free(c->slots);
    dev_free(c->bar);
    dev_free(c->gsnap);
    dev_free(c->seeds);
    dev_free(c->btab);
    dev_free(c->qseeds);
    dev_free(c->b_counters);
    dev_free(c->sacc);
    dev_free(c->scen);
    dev_free(c->scen32);
    dev_free(c->scnt);
    dev_free(c->scounters);
    dev_free(c->sslab);
    dev_free(c->slsum);
    dev_free(c->mbuf);
    if (c->own_net) mf4d_net_destroy(c->own_net);
    c->own_net = nullptr;
    if (c->h_scounters) (void)hipHostFree(c->h_scounters);
    {
        char* st = static_cast<char*>(c->staging);
        dev_free(st);
        c->staging = nullptr;
    }
    if (c->side) (void)hipStreamDestroy(c->side);
    for (hipEvent_t e : {c->ev_labels, c->ev_pread, c->ev_chunk, c->ev_stat, c->ev_read[0], c->ev_read[1], c->ev_issue})
        if (e) (void)hipEventDestroy(e);
    c->h_counters = nullptr;  // inside h_stat
    if (c->h_stat) (void)hipHostFree(c->h_stat);
    for (int i = 0; i < 4; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    for (int i = 0; i < 16; ++i)
        if (c->rev[i]) (void)hipEventDestroy(c->rev[i]);
    delete c;
}

int mf4d_set_tile(mf4d_ctx* c, int bt) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    settle_submit(c);  // a submitted grow first
    if (bt != 4 && bt != 8 && bt != 16) return fail(MF4D_ERR_ARG, "tile t-extent %d not in {4,8,16}", bt);
    if (c->has_field) return fail(MF4D_ERR_STATE, "tile shape must be set before the field is loaded");
    c->bt = bt;
    return MF4D_OK;
}

int mf4d_load_field(mf4d_ctx* c, const float* field, int X, int Y, int Z, int T, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
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
    if (g.NZt > 65535 || T > 65535)
        return fail(MF4D_ERR_UNSUPPORTED, "Z/8 and T must stay within a 65535 grid dimension");
    if (g.nwords * 32ull >= (1ull << 32) || (uint64_t)X * Y * Z * T >= (1ull << 32) - 1)
        return fail(MF4D_ERR_UNSUPPORTED, "grid of %llu voxel-steps (padded %llu) needs >= 2^32 bits",
                    (unsigned long long)X * Y * Z * T, (unsigned long long)g.nwords * 32ull);
    g.NT = (uint32_t)nt;
    g.WCAP = (uint32_t)((nt + kWorkSubs - 1) / kWorkSubs);
    HIP_TRY(hipSetDevice(c->device));
    free_particles(c);
    free_field(c);
    c->state = 0;
    const size_t V = (size_t)X * Y * Z * T;
    int rc = dev_alloc(&c->field, V);
    if (!rc) rc = dev_alloc(&c->Af, g.nwords);
    if (!rc) rc = dev_alloc(&c->Lf, g.nwords);
    if (!rc) rc = dev_alloc(&c->active, (size_t)g.NT + 8);
    if (!rc) rc = dev_alloc(&c->dirty, 2 * (size_t)g.NT);
    if (!rc) rc = dev_alloc(&c->chg, 2 * (size_t)g.NT + 8);
    if (!rc) rc = dev_alloc(&c->work, 2 * (size_t)kWorkSubs * g.WCAP);
    if (!rc) rc = dev_alloc(&c->wcnt, 2 * (size_t)kWorkSubs * kWcntStride);
    if (!rc) rc = dev_alloc(&c->tsum, (size_t)g.NT);
    if (!rc) rc = dev_alloc(&c->cand, (size_t)g.NT);
    const BrickDims bd{T, (Z + 7) / 8, (Y + 7) / 8, (X + 7) / 8};
    const size_t nbricks = (size_t)bd.T * bd.D * bd.H * bd.W;
    if (!rc) rc = dev_alloc(&c->bstats, nbricks);
    if (!rc) rc = dev_alloc(&c->feat, nbricks * 16);
    if (!rc) rc = dev_alloc(&c->blogits, nbricks);
    if (!rc) rc = dev_alloc(&c->tpred, (size_t)g.NT);
    if (rc) {
        free_field(c);
        return rc;
    }
    HIP_TRY(hipMemcpyAsync(c->field, field, V * sizeof(float),
                           where == MF4D_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                           c->stream));
    launch_fill_u32(c->Af, 0, g.nwords, c->stream);
    launch_fill_u32(c->Lf, 0, g.nwords, c->stream);
    launch_summaries(g, c->field, c->tsum, c->stream);
    c->bstats_valid = false;
    rc = sync(c);
    if (rc) {
        free_field(c);
        return rc;
    }
    c->g = g;
    c->bd = bd;
    c->has_field = true;
    return MF4D_OK;
}

int mf4d_load_particles(mf4d_ctx* c, const float* xyz, const float* attr, int64_t P, int T,
                        int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->has_field) return fail(MF4D_ERR_STATE, "load the field before the particles");
    if (P > 0 && T != c->g.T) return fail(MF4D_ERR_ARG, "particle T %d differs from field T %d", T, c->g.T);
    return mf4d_load_particles_rate(c, xyz, attr, P, c->g.T, 1, where);
}

int mf4d_load_particles_rate(mf4d_ctx* c, const float* xyz, const float* attr, int64_t P, int Tp,
                             int steps_per_field_step, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (!c->has_field) return fail(MF4D_ERR_STATE, "load the field before the particles");
    if (P < 0) return fail(MF4D_ERR_ARG, "P < 0");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    if (P > 0 && (!xyz || !attr)) return fail(MF4D_ERR_ARG, "xyz or attr is NULL");
    const int r = steps_per_field_step;
    if (r < 1 || r > 1024) return fail(MF4D_ERR_ARG, "steps per field step %d not in 1..1024", r);
    if (P > 0 && (Tp < 1 || (int64_t)Tp > (int64_t)r * c->g.T))
        return fail(MF4D_ERR_ARG, "%d particle steps at %d per field step do not fit %d field steps", Tp, r,
                    c->g.T);
    PGeom pg{};
    pg.P = P;
    pg.T = Tp;
    pg.tr = r;
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
    if (!rc) rc = dev_alloc(&c->clist, Q);
    if (!rc) rc = dev_alloc(&c->pdirty, (size_t)(P + 31) / 32);
    if (!rc) rc = dev_alloc(&c->pflag, (size_t)P);
    if (!rc) rc = dev_alloc(&c->dlist, (size_t)P);
    if (!rc) rc = dev_alloc(&c->psum, (size_t)P);
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
            dev_free(tmp);
            free_particles(c);
            return fail(MF4D_ERR_HIP, "particle upload failed: %s", hipGetErrorString(e));
        }
        dx = tmp;
        da = tmp + nxyz;
    }
    launch_bin_particles(c->g, pg, dx, da, c->bins, c->attr_t, c->stream);
    launch_particle_summaries(pg, c->attr_t, c->psum, c->stream);
    c->bstats_valid = false;
    launch_fill_u32(c->pdirty, 0, (P + 31) / 32, c->stream);
    // the clustering reads positions and values as loaded: keep the upload
    // buffer, or copy device inputs into one laid out the same way
    if (tmp) {
        c->praw = tmp;
        tmp = nullptr;
    } else {
        rc = dev_alloc(&c->praw, nxyz + nat);
        if (!rc) {
            hipError_t e = hipMemcpyAsync(c->praw, xyz, nxyz * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->praw + nxyz, attr, nat * sizeof(float), hipMemcpyDeviceToDevice,
                                   c->stream);
            if (e != hipSuccess) rc = fail(MF4D_ERR_HIP, "particle copy failed: %s", hipGetErrorString(e));
        }
    }
    if (!rc) rc = sync(c);
    dev_free(tmp);
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
    settle_submit(c);  // a submitted grow first
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
    settle_submit(c);  // a submitted grow first
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
    settle_submit(c);  // a submitted grow first
    if (cap < 0) return fail(MF4D_ERR_ARG, "cap < 0");
    c->max_rounds = cap;
    return MF4D_OK;
}

int mf4d_set_admit_mode(mf4d_ctx* c, int mode) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    settle_submit(c);  // a submitted grow first
    if (mode != MF4D_ADMIT_TILES && mode != MF4D_ADMIT_ALL)
        return fail(MF4D_ERR_ARG, "unknown admissibility mode %d", mode);
    c->admit_all = mode == MF4D_ADMIT_ALL;
    return MF4D_OK;
}

int mf4d_set_trajectory_mode(mf4d_ctx* c, int mode) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    settle_submit(c);  // a submitted grow first
    if (mode != MF4D_TRAJ_BOTH && mode != MF4D_TRAJ_FORWARD)
        return fail(MF4D_ERR_ARG, "unknown trajectory mode %d", mode);
    c->forward_only = mode == MF4D_TRAJ_FORWARD;
    c->state = 0;  // labels of an earlier grow no longer describe this mode
    return MF4D_OK;
}

int mf4d_set_phase_timing(mf4d_ctx* c, int on) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    settle_submit(c);  // a submitted grow first
    if (on != 0 && on != 1) return fail(MF4D_ERR_ARG, "on must be 0 or 1");
    c->phase_timing = on == 1;
    return MF4D_OK;
}

int mf4d_set_schedule(mf4d_ctx* c, int mode) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    settle_submit(c);  // a submitted grow first
    if (mode != MF4D_SCHED_PERSISTENT && mode != MF4D_SCHED_LAUNCH && mode != MF4D_SCHED_JACOBI)
        return fail(MF4D_ERR_ARG, "unknown schedule %d", mode);
    c->schedule = mode;
    return MF4D_OK;
}

// Brick statistics (network input) of the loaded field and particles, on the
// context's stream; computed once per load, when first needed.
static void ensure_brick_stats(mf4d_ctx* c) {
    if (c->bstats_valid) return;
    launch_brick_stats(c->g, c->has_particles ? c->pg : PGeom{}, c->bd, c->field,
                       c->has_particles ? c->bins : nullptr, c->bstats, c->stream);
    c->bstats_valid = true;
}

// Buffers of the score-ordered schedulers (sized by the tile count).
static int ensure_priority(mf4d_ctx* c) {
    if (c->pr_buf) return MF4D_OK;
    const uint32_t NT = c->g.NT;
    int rc = dev_alloc(&c->pr_buf, 4 * (size_t)NT + 1);
    if (rc) return rc;
    size_t bytes = 0;
    HIP_TRY(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, bytes, c->pr_buf, c->pr_buf + 2 * (size_t)NT,
                                                         c->pr_buf + NT, c->pr_buf + 3 * (size_t)NT, (int)NT, 0,
                                                         32, c->stream));
    char* tmp = nullptr;
    rc = dev_alloc(&tmp, bytes);
    if (rc) {
        dev_free(c->pr_buf);
        return rc;
    }
    c->pr_tmp = tmp;
    c->pr_tmp_bytes = bytes;
    return MF4D_OK;
}

// The verification round after the rounds converged (run as launches
// whatever the schedule), then plain rounds while it found work.
static int verify_round(mf4d_ctx* c, const Dev& d, int64_t* rounds) {
    c->stats_ready = false;
    const int par = (int)(c->round & 1);
    launch_verify_schedule(d, par, c->stream);
    Dev dv = d;
    dv.pull_all = 1;
    launch_fill_u32(c->counters + C_ROUNDS, 0, 1, c->stream);
    launch_round(dv, c->round, c->stream);
    launch_work_total(d, par ^ 1, c->stream);
    int rc = read_counters(c);
    if (rc) return rc;
    c->round += c->h_counters[C_ROUNDS];
    *rounds = c->h_counters[C_ROUNDS];
    if (c->h_counters[C_NWORK0 + (par ^ 1)] == 0) return MF4D_OK;
    int64_t more = 0;
    rc = run_rounds(c, d, &more);
    *rounds += more;
    return rc;
}

// A fresh grow; with rd_f / rd_p set, their read-outs are queued behind the
// rounds where the schedule allows it (reads_done then reports whether they
// ran on the final labels).
// A grow in two halves around its rounds: grow_begin queues the reset,
// admissibility, seeding and (score-ordered) the priority pass; grow_end
// runs the verification round, takes the statistics and marks the labels.
struct GrowRun {
    Dev d;
    bool ordered;
};

static int grow_begin(mf4d_ctx* c, GrowRun* gr) {
    if (!c->has_field) return fail(MF4D_ERR_STATE, "no field loaded");
    if (!c->has_crit) return fail(MF4D_ERR_STATE, "no criteria set");
    HIP_TRY(hipSetDevice(c->device));
    if (c->async_grow) {
        // the read-outs of the grow before are deferred (or still run) on
        // the current set: grow on the other one (allocated on first use),
        // once its own read-outs are done
        int rc = MF4D_OK;
        if (c->dread.valid && c->dread.set != c->lset) rc = issue_deferred(c, nullptr, false);  // on that set
        if (rc) return rc;
        if (!c->Lf_alt) rc = dev_alloc(&c->Lf_alt, c->g.nwords);
        if (!rc && !c->active_alt) rc = dev_alloc(&c->active_alt, (size_t)c->g.NT + 8);
        if (!rc && c->has_particles && !c->Lp_alt) rc = dev_alloc(&c->Lp_alt, (size_t)c->pg.P * c->pg.W);
        if (!rc && c->has_particles && !c->pflag_alt) rc = dev_alloc(&c->pflag_alt, (size_t)c->pg.P);
        if (rc) return rc;
        if (!c->alt_ready) {  // labels outside this grow's candidates read as cleared
            launch_fill_u32(c->Lf_alt, 0u, c->g.nwords, c->stream);
            if (c->has_particles)
                launch_fill_u32(reinterpret_cast<uint32_t*>(c->Lp_alt), 0u, 2ull * (uint64_t)c->pg.P * c->pg.W,
                                c->stream);
            c->alt_ready = true;
        }
        std::swap(c->Lf, c->Lf_alt);
        std::swap(c->active, c->active_alt);
        if (c->has_particles) {
            std::swap(c->Lp, c->Lp_alt);
            std::swap(c->pflag, c->pflag_alt);
        }
        c->lset ^= 1;
        if (c->read_pending[c->lset]) {
            HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_read[c->lset], 0));
            c->read_pending[c->lset] = false;
        }
    } else {
        int rc = settle_async(c);
        if (rc) return rc;
    }
    hipStream_t s = c->stream;
    const Dev d = make_dev(c);
    c->state = 0;
    c->round = 0;
    c->ms_phase[0] = c->ms_phase[1] = c->ms_phase[2] = 0;
    c->members_pending[0] = c->members_pending[1] = false;
    launch_reset(d, s);
    c->timed = c->phase_timing;
    if (c->timed) HIP_TRY(hipEventRecord(c->ev[0], s));
    Dev dp = d;
    const bool ordered = c->priority != MF4D_SCHEDULER_PLAIN && !d.admit_all;
    const bool predicted = c->net && !d.admit_all;
    if (predicted) {
        // the predictor marks the candidate tiles to test before the rounds
        ensure_brick_stats(c);
        launch_features(c->bd, c->bstats, c->crit[0], c->feat, s);
        int rc = net_infer(c->net, c->feat, c->bd.T, c->bd.D, c->bd.H, c->bd.W, c->blogits, s);
        if (rc) return fail(rc, "predictor: %s", net_last_error());
        launch_tile_predict(c->g, c->bd, c->blogits, c->pred_thr, c->tpred, s);
        dp.tpred = c->tpred;
    }
    uint32_t* plist = nullptr;
    uint32_t* pcount = nullptr;
    if (ordered) {
        // priority list: candidate tiles in descending score, scored by the
        // network (learned) or by their greatest field value (heuristic)
        int rc = ensure_priority(c);
        if (rc) return rc;
        const uint32_t NT = c->g.NT;
        uint32_t* keys = c->pr_buf;
        uint32_t* vals = c->pr_buf + NT;
        uint32_t* skeys = c->pr_buf + 2 * (size_t)NT;
        plist = c->pr_buf + 3 * (size_t)NT;
        pcount = c->pr_buf + 4 * (size_t)NT;
        launch_fill_u32(pcount, 0, 1, s);
        const bool learned = c->priority == MF4D_SCHEDULER_LEARNED && c->net;
        launch_priority_keys(d, learned ? c->blogits : nullptr, c->bd.W, c->bd.H, c->bd.D,
                             learned ? c->pred_thr : -INFINITY, keys, vals, pcount, s);
        size_t bytes = c->pr_tmp_bytes;
        HIP_TRY(hipcub::DeviceRadixSort::SortPairsDescending(c->pr_tmp, bytes, keys, skeys, vals, plist, (int)NT,
                                                             0, 32, s));
    }
    launch_admit_field(dp, s);
    if (c->timed) HIP_TRY(hipEventRecord(c->ev[1], s));
    launch_admit_particles(d, s);
    if (c->timed) HIP_TRY(hipEventRecord(c->ev[2], s));
    launch_seeds(d, c->seeds, c->S, s);
    if (c->async_grow && c->dread.valid && (c->schedule != MF4D_SCHED_LAUNCH || c->issue_round == 0)) {
        // the grow before's read-outs, beside this grow's rounds (after its
        // admissibility passes, the bandwidth-heavy part; with launched
        // rounds after the first issue_round rounds, whose sweeps iterate
        // longest)
        HIP_TRY(hipEventRecord(c->ev_issue, s));
        int rc = issue_deferred(c, c->ev_issue, false);
        if (rc) return rc;
    }
    if (ordered) launch_priority_sweep(d, plist, pcount, c->pr_waves, s);
    gr->d = d;
    gr->ordered = ordered;
    return MF4D_OK;
}

static int grow_end(mf4d_ctx* c, const GrowRun& gr, int64_t rounds, mf4d_stats* out) {
    const Dev& d = gr.d;
    int rc = MF4D_OK;
    int64_t verify_rounds = 0;
    if (gr.ordered && c->state == 1) {
        // verification round: every tile holding an admissible voxel-step is
        // swept and every coupled particle-step pulled; should anything
        // change, the plain rounds continue until nothing does
        rc = verify_round(c, d, &verify_rounds);
        if (rc) return rc;
    }
    if (c->state == 1) c->last_rounds = rounds;
    if (c->timed) HIP_TRY(hipEventRecord(c->ev[3], c->stream));
    rc = finish_stats(c, out, true, rounds + verify_rounds);
    if (rc) return rc;
    c->stats.verify_rounds = verify_rounds;
    if (out) *out = c->stats;
    mark_labels(c);
    if (c->state == 2) return fail(MF4D_ERR_NOT_CONVERGED, "stopped after %lld rounds", (long long)rounds);
    return MF4D_OK;
}

static int grow_impl(mf4d_ctx* c, mf4d_stats* out) {
    GrowRun gr;
    int rc = grow_begin(c, &gr);
    if (rc) return rc;
    int64_t rounds = 0;
    rc = run_rounds(c, gr.d, &rounds);
    if (rc) return rc;
    return grow_end(c, gr, rounds, out);
}

int mf4d_grow(mf4d_ctx* c, mf4d_stats* out) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    c->rd_f = nullptr;
    c->rd_p = nullptr;
    return grow_impl(c, out);
}

int mf4d_set_read_async(mf4d_ctx* c, int on) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    HIP_TRY(hipSetDevice(c->device));
    int rc = settle_async(c);
    if (rc) return rc;
    c->read_async = on != 0;
    return MF4D_OK;
}

int mf4d_read_wait(mf4d_ctx* c) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    HIP_TRY(hipSetDevice(c->device));
    return settle_async(c);
}

}  // extern "C"

namespace {

int check_read_buffers(mf4d_ctx* c, const uint32_t* field_dst, size_t nwords, const uint8_t* particle_dst,
                       size_t n) {
    if (!c->has_field) return fail(MF4D_ERR_STATE, "no field loaded");
    if (particle_dst && !c->has_particles) return fail(MF4D_ERR_STATE, "no particles loaded");
    const uint64_t V = (uint64_t)c->g.X * c->g.Y * c->g.Z * c->g.T;
    if (field_dst && nwords < (V + 31) / 32)
        return fail(MF4D_ERR_ARG, "field_dst holds %zu words, %llu needed", nwords, (unsigned long long)((V + 31) / 32));
    if (particle_dst && n < (size_t)c->pg.P * c->pg.T)
        return fail(MF4D_ERR_ARG, "particle_dst holds %zu bytes, %zu needed", n, (size_t)c->pg.P * c->pg.T);
    return MF4D_OK;
}

// Read-outs queued behind the rounds only where the labels are final when
// the rounds end: not with a verification round (score-ordered schedulers),
// Jacobi sweeps or phase timing (events per round).
bool reads_can_queue(const mf4d_ctx* c) {
    const bool ordered = c->priority != MF4D_SCHEDULER_PLAIN && !c->admit_all;
    return !ordered && !c->phase_timing && c->schedule != MF4D_SCHED_JACOBI;
}

// After a grow whose read-outs were queued behind its rounds (rc: the
// grow's status): where they did not run on the final labels, read out now.
int finish_grow_read(mf4d_ctx* c, int rc, uint32_t* field_dst, size_t nwords, uint8_t* particle_dst, size_t n) {
    const bool done = c->reads_done;
    c->rd_f = nullptr;
    c->rd_p = nullptr;
    c->reads_done = false;
    if (rc != MF4D_OK && rc != MF4D_ERR_NOT_CONVERGED) return rc;
    // the masks are those of the labels as they stand, converged or not
    if (done) {
        c->members_pending[0] = field_dst != nullptr;
        c->members_pending[1] = particle_dst != nullptr;
    } else {
        if (field_dst) {
            int r2 = mf4d_read_field_mask(c, field_dst, nwords, MF4D_DEVICE);
            if (r2) return r2;
        }
        if (particle_dst) {
            int r2 = mf4d_read_particle_mask(c, particle_dst, n, MF4D_DEVICE);
            if (r2) return r2;
        }
    }
    if (rc == MF4D_ERR_NOT_CONVERGED) return fail(rc, "stopped after %lld rounds", (long long)c->stats.rounds);
    return MF4D_OK;
}

// The rest of a submitted grow: wait for its first chunk, run the rounds it
// still needs, take its statistics and read out where needed.
int complete_submitted(mf4d_ctx* c, mf4d_stats* out) {
    c->submitted = 0;
    HIP_TRY(hipSetDevice(c->device));
    const GrowRun gr{c->sub_d, false};
    const RoundChunk ch{c->sub_chunk, c->sub_npar};
    int64_t rounds = 0;
    int rc = run_rounds(c, gr.d, &rounds, &ch);
    if (!rc) rc = grow_end(c, gr, rounds, out);
    return finish_grow_read(c, rc, c->sub_f, c->sub_nwords, c->sub_p, c->sub_n);
}

// Any call on a context with a submitted grow completes that grow first and
// keeps its result for mf4d_grow_finish.
int settle_submit(mf4d_ctx* c) {
    if (c->submitted != 2) return MF4D_OK;
    c->sub_rc = complete_submitted(c, &c->sub_stats);
    c->sub_err = c->sub_rc ? std::string(mf4d_last_error()) : std::string();
    c->submitted = 1;
    return MF4D_OK;
}

}  // namespace

extern "C" {

int mf4d_grow_read(mf4d_ctx* c, uint32_t* field_dst, size_t nwords, uint8_t* particle_dst, size_t n,
                   mf4d_stats* out) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    settle_submit(c);
    int rc = check_read_buffers(c, field_dst, nwords, particle_dst, n);
    if (rc) return rc;
    const bool queue = reads_can_queue(c);
    if (queue && c->read_async) {
        // asynchronous: the read-outs are deferred (issued beside the next
        // asynchronous grow_read's rounds, or by the next other call) and read
        // the labels as this grow leaves them, converged or not
        c->async_grow = true;
        rc = grow_impl(c, out);
        c->async_grow = false;
        if (rc != MF4D_OK && rc != MF4D_ERR_NOT_CONVERGED) return rc;
        c->dread.f = field_dst;
        c->dread.p = particle_dst;
        c->dread.set = c->lset;
        c->dread.valid = field_dst || particle_dst;
        if (rc == MF4D_ERR_NOT_CONVERGED) return fail(rc, "stopped after %lld rounds", (long long)c->stats.rounds);
        return MF4D_OK;
    }
    c->rd_f = queue ? field_dst : nullptr;
    c->rd_p = queue ? particle_dst : nullptr;
    c->reads_done = false;
    rc = grow_impl(c, out);
    return finish_grow_read(c, rc, field_dst, nwords, particle_dst, n);
}

int mf4d_grow_submit(mf4d_ctx* c, uint32_t* field_dst, size_t nwords, uint8_t* particle_dst, size_t n) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (c->submitted) return fail(MF4D_ERR_STATE, "a submitted grow awaits mf4d_grow_finish");
    int rc = check_read_buffers(c, field_dst, nwords, particle_dst, n);
    if (rc) return rc;
    if (!reads_can_queue(c) || c->schedule != MF4D_SCHED_LAUNCH) {
        // the whole grow now; its result waits for mf4d_grow_finish
        c->sub_rc = mf4d_grow_read(c, field_dst, nwords, particle_dst, n, &c->sub_stats);
        c->sub_err = c->sub_rc ? std::string(mf4d_last_error()) : std::string();
        c->submitted = 1;
        return MF4D_OK;
    }
    HIP_TRY(hipSetDevice(c->device));
    rc = settle_async(c);
    if (rc) return rc;
    c->rd_f = field_dst;
    c->rd_p = particle_dst;
    c->reads_done = false;
    GrowRun gr;
    rc = grow_begin(c, &gr);
    RoundChunk ch{0, 0};
    if (!rc) rc = queue_chunk(c, gr.d, 0, &ch);
    if (rc) {
        c->rd_f = nullptr;
        c->rd_p = nullptr;
        return rc;
    }
    c->sub_d = gr.d;
    c->sub_chunk = ch.n;
    c->sub_npar = ch.npar;
    c->sub_f = field_dst;
    c->sub_nwords = nwords;
    c->sub_p = particle_dst;
    c->sub_n = n;
    c->submitted = 2;
    return MF4D_OK;
}

int mf4d_grow_finish(mf4d_ctx* c, mf4d_stats* out) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->submitted) return fail(MF4D_ERR_STATE, "no submitted grow");
    if (c->submitted == 2) return complete_submitted(c, out);
    c->submitted = 0;
    if (out) *out = c->sub_stats;
    if (c->sub_rc) return fail(c->sub_rc, "%s", c->sub_err.c_str());
    return MF4D_OK;
}

int mf4d_grow_resume(mf4d_ctx* c, mf4d_stats* out) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (c->state != 2) return fail(MF4D_ERR_STATE, "nothing to resume");
    HIP_TRY(hipSetDevice(c->device));
    const Dev d = make_dev(c);
    if (c->timed) HIP_TRY(hipEventRecord(c->ev[2], c->stream));
    int64_t rounds = 0;
    int rc = run_rounds(c, d, &rounds);
    if (rc) return rc;
    if (c->timed) HIP_TRY(hipEventRecord(c->ev[3], c->stream));
    rc = finish_stats(c, out, false, rounds);
    if (rc) return rc;
    mark_labels(c);
    if (c->state == 2) return fail(MF4D_ERR_NOT_CONVERGED, "stopped after %lld more rounds", (long long)rounds);
    return MF4D_OK;
}

int mf4d_reset_labels(mf4d_ctx* c) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (!c->has_field) return fail(MF4D_ERR_STATE, "no field loaded");
    HIP_TRY(hipSetDevice(c->device));
    launch_fill_u32(c->Lf, 0u, c->g.nwords, c->stream);
    if (c->has_particles && c->Lp)
        launch_fill_u32(reinterpret_cast<uint32_t*>(c->Lp), 0u, 2ull * (uint64_t)c->pg.P * c->pg.W, c->stream);
    int rc = sync(c);
    if (rc) return rc;
    c->state = 0;
    c->round = 0;
    mark_labels(c);
    return MF4D_OK;
}

// Member counts folded on the device by stream-ordered reads: copy them to
// the host (once, when asked for) and record them.
static int settle_members(mf4d_ctx* c) {
    if (!c->members_pending[0] && !c->members_pending[1]) return MF4D_OK;
    HIP_TRY(hipMemcpyAsync(c->h_stat + S_MEMBERS_F, c->stat64 + S_MEMBERS_F, 2 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, c->stream));
    int rc = sync(c);
    if (rc) return rc;
    if (c->members_pending[0]) c->stats.members_field = (int64_t)c->h_stat[S_MEMBERS_F];
    if (c->members_pending[1]) c->stats.members_particle = (int64_t)c->h_stat[S_MEMBERS_P];
    c->members_pending[0] = c->members_pending[1] = false;
    return MF4D_OK;
}

int mf4d_read_field_mask(mf4d_ctx* c, uint32_t* dst, size_t nwords, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
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
    launch_read_field(make_dev(c), out, c->stream);
    launch_fold_slots(make_dev(c), SL_MEMBERS_F, S_MEMBERS_F, c->stream, true);
    if (where == MF4D_HOST)
        HIP_TRY(hipMemcpyAsync(dst, out, need * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    c->members_pending[0] = true;  // the count stays on the device until asked for
    if (where == MF4D_DEVICE) return MF4D_OK;  // stream-ordered
    return settle_members(c);
}

int mf4d_read_particle_mask(mf4d_ctx* c, uint8_t* dst, size_t n, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
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
    // Into a device buffer the read-out runs on the side stream, after the
    // last work that changed the labels and beside whatever the context
    // stream does meanwhile (the field read-out); the context stream then
    // waits for it, so the call stays ordered on that stream.
    const bool side = where == MF4D_DEVICE && c->labels_marked;
    hipStream_t rs = side ? c->side : c->stream;
    if (side) HIP_TRY(hipStreamWaitEvent(c->side, c->ev_labels, 0));
    launch_read_particles(make_dev(c), out, rs);
    launch_fold_slots(make_dev(c), SL_MEMBERS_P, S_MEMBERS_P, rs, true);
    if (where == MF4D_HOST)
        HIP_TRY(hipMemcpyAsync(dst, out, need, hipMemcpyDeviceToHost, c->stream));
    if (side) {
        HIP_TRY(hipEventRecord(c->ev_pread, c->side));
        HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_pread, 0));
    }
    c->members_pending[1] = true;  // the count stays on the device until asked for
    if (where == MF4D_DEVICE) return MF4D_OK;  // stream-ordered
    return settle_members(c);
}

int mf4d_read_particle_segments(mf4d_ctx* c, uint8_t* dst, size_t n, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
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
    launch_particle_segments(make_dev(c), out, c->stream);
    if (where == MF4D_HOST)
        HIP_TRY(hipMemcpyAsync(dst, out, need, hipMemcpyDeviceToHost, c->stream));
    if (where == MF4D_DEVICE) return MF4D_OK;  // stream-ordered
    return sync(c);
}

int mf4d_grow_seed_ids(mf4d_ctx* c, int32_t* field_ids, size_t nf, int32_t* particle_ids, size_t np,
                       int where, int64_t* grows) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (!c->has_field) return fail(MF4D_ERR_STATE, "no field loaded");
    if (!c->has_crit) return fail(MF4D_ERR_STATE, "no criteria set");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    const Geom& g = c->g;
    const size_t V = (size_t)g.X * g.Y * g.Z * g.T;
    const int64_t P = c->has_particles ? c->pg.P : 0;
    const size_t Qp = P > 0 ? (size_t)P * c->pg.T : 0;
    if (!field_ids || nf < V) return fail(MF4D_ERR_ARG, "field ids need %zu elements", V);
    const bool want_p = P > 0 && particle_ids;
    if (want_p && np < Qp) return fail(MF4D_ERR_ARG, "particle ids need %zu elements", Qp);
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int64_t S = c->S;
    std::vector<int32_t> hs((size_t)S * 4);
    if (S > 0) HIP_TRY(hipMemcpy(hs.data(), c->seeds, hs.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    int32_t* fo = field_ids;
    int32_t* po = want_p ? particle_ids : nullptr;
    if (where == MF4D_HOST) {
        void* st = nullptr;
        int rc = staging_for(c, (V + (want_p ? Qp : 0)) * sizeof(int32_t), &st);
        if (rc) return rc;
        fo = (int32_t*)st;
        po = want_p ? fo + V : nullptr;
    }
    // canonical member words of one grow, and the members seen so far
    struct Scratch {
        uint32_t* words = nullptr;
        uint32_t* seen_f = nullptr;
        unsigned long long* seen_p = nullptr;
        ~Scratch() { dev_free(words); dev_free(seen_f); dev_free(seen_p); }
    } sc;
    const size_t nw = (V + 31) / 32, pw = P > 0 ? (size_t)(c->pg.T + 63) / 64 : 0;
    int rc = dev_alloc(&sc.words, nw);
    if (!rc) rc = dev_alloc(&sc.seen_f, nw);
    if (!rc && po) rc = dev_alloc(&sc.seen_p, (size_t)P * pw);
    if (rc) return rc;
    launch_fill_u32((uint32_t*)fo, 0xFFFFFFFFu, V, s);
    launch_fill_u32(sc.seen_f, 0u, nw, s);
    if (po) {
        launch_fill_u32((uint32_t*)po, 0xFFFFFFFFu, Qp, s);
        launch_fill_u32((uint32_t*)sc.seen_p, 0u, 2 * (size_t)P * pw, s);
    }
    int32_t* const all_seeds = c->seeds;
    int64_t ngrow = 0;
    for (int64_t i = 0; i < S; ++i) {
        const int32_t* sd = &hs[(size_t)i * 4];
        const size_t v = (((size_t)sd[3] * g.Z + sd[2]) * g.Y + sd[1]) * g.X + sd[0];
        // a seed inside an earlier seed's region reaches nothing new (every
        // node it reaches, that region reaches); an inadmissible one is dropped
        int32_t cur = 0;
        float fv = 0.0f;
        HIP_TRY(hipMemcpyAsync(&cur, fo + v, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&fv, c->field + v, sizeof(float), hipMemcpyDeviceToHost, s));
        rc = sync(c);
        if (rc) return rc;
        if (cur != -1 || !(c->crit[0] <= fv && fv <= c->crit[1])) continue;
        c->seeds = all_seeds + 4 * i;
        c->S = 1;
        rc = mf4d_grow(c, nullptr);
        c->seeds = all_seeds;
        c->S = S;
        if (rc) {
            c->state = 0;
            return rc;
        }
        ++ngrow;
        const Dev d = make_dev(c);
        launch_read_field(d, sc.words, s);
        launch_fold_slots(d, SL_MEMBERS_F, S_MEMBERS_F, s, true);  // clears the member slots
        launch_seed_ids(d, sc.words, sc.seen_f, sc.seen_p, (int32_t)i, fo, po, s);
    }
    c->state = 0;  // the labels hold the last single-seed grow, not the seeds' union
    if (where == MF4D_HOST) {
        HIP_TRY(hipMemcpyAsync(field_ids, fo, V * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (po) HIP_TRY(hipMemcpyAsync(particle_ids, po, Qp * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    rc = sync(c);
    if (rc) return rc;
    if (grows) *grows = ngrow;
    return MF4D_OK;
}

int mf4d_set_queries(mf4d_ctx* c, int Q, const float* crit, const int32_t* qxyzt, int64_t S,
                     int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (!c->has_field) return fail(MF4D_ERR_STATE, "load the field before the queries");
    if (Q < 1 || Q > 256) return fail(MF4D_ERR_ARG, "Q = %d not in 1..256", Q);
    if (!crit || S < 0 || (S > 0 && !qxyzt)) return fail(MF4D_ERR_ARG, "bad query arrays");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    if (S > (1ll << 30)) return fail(MF4D_ERR_UNSUPPORTED, "too many seeds");
    HIP_TRY(hipSetDevice(c->device));
    std::vector<float> cr((size_t)Q * 4);
    std::vector<int32_t> sd((size_t)S * 5);
    const hipMemcpyKind k = where == MF4D_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
    HIP_TRY(hipMemcpy(cr.data(), crit, cr.size() * sizeof(float), k));
    if (S > 0) HIP_TRY(hipMemcpy(sd.data(), qxyzt, sd.size() * sizeof(int32_t), k));
    for (float v : cr)
        if (v != v) return fail(MF4D_ERR_ARG, "a query bound is NaN");
    for (int64_t i = 0; i < S; ++i) {
        const int32_t* q = &sd[i * 5];
        if (q[0] < 0 || q[0] >= c->g.X || q[1] < 0 || q[1] >= c->g.Y || q[2] < 0 ||
            q[2] >= c->g.Z || q[3] < 0 || q[3] >= c->g.T)
            return fail(MF4D_ERR_RANGE, "query seed %lld outside the grid", (long long)i);
        if (q[4] < 0 || q[4] >= Q)
            return fail(MF4D_ERR_RANGE, "query seed %lld names query %d of %d", (long long)i, q[4], Q);
    }
    // sorted bounds and prefix masks: {q : lo_q <= v} is a prefix of the
    // ascending order of lo, {q : hi_q >= v} a prefix of the descending order
    std::vector<float> tab(kTabWords, 0.0f);
    uint32_t* masks = reinterpret_cast<uint32_t*>(tab.data() + 1024);
    for (int type = 0; type < 2; ++type) {
        for (int side = 0; side < 2; ++side) {
            std::vector<int> order(Q);
            for (int q = 0; q < Q; ++q) order[q] = q;
            const int col = type * 2 + side;
            if (side == 0)
                std::stable_sort(order.begin(), order.end(),
                                 [&](int a, int b) { return cr[a * 4 + col] < cr[b * 4 + col]; });
            else
                std::stable_sort(order.begin(), order.end(),
                                 [&](int a, int b) { return cr[a * 4 + col] > cr[b * 4 + col]; });
            float* sorted = tab.data() + 256 * col;
            uint32_t* m = masks + col * 257 * 8;
            for (int i = 0; i < Q; ++i) sorted[i] = cr[order[i] * 4 + col];
            for (int i = 0; i < Q; ++i) {
                for (int w = 0; w < 8; ++w) m[(i + 1) * 8 + w] = m[i * 8 + w];
                m[(i + 1) * 8 + (order[i] >> 5)] |= 1u << (order[i] & 31);
            }
        }
    }
    if (!c->btab) {
        int rc = dev_alloc(&c->btab, (size_t)kTabWords);
        if (rc) return rc;
    }
    if (S > c->qseeds_cap) {
        int32_t* ns = nullptr;
        int rc = dev_alloc(&ns, (size_t)S * 5);
        if (rc) return rc;
        dev_free(c->qseeds);
        c->qseeds = ns;
        c->qseeds_cap = S;
    }
    HIP_TRY(hipMemcpy(c->btab, tab.data(), kTabWords * sizeof(float), hipMemcpyHostToDevice));
    if (S > 0)
        HIP_TRY(hipMemcpy(c->qseeds, sd.data(), sd.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    c->Q = Q;
    c->QS = S;
    c->b_grown = false;
    return MF4D_OK;
}

int mf4d_set_batched_tile(mf4d_ctx* c, int bx, int by, int bz, int bt) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    settle_submit(c);  // a submitted grow first
    const int e[4] = {bx, by, bz, bt};
    int lg[4];
    for (int i = 0; i < 4; ++i) {
        lg[i] = e[i] > 0 ? ilog2(e[i]) : -1;
        if (lg[i] < 0 || e[i] > 64) return fail(MF4D_ERR_ARG, "tile extents must be powers of two <= 64");
    }
    if (bx * by * bz * bt != 512) return fail(MF4D_ERR_ARG, "a batched tile holds 512 voxel-steps");
    for (int i = 0; i < 4; ++i) c->blog[i] = lg[i];
    dev_free(c->b_active);
    dev_free(c->b_dirty);
    dev_free(c->b_chg);
    dev_free(c->b_work);
    c->NTB = 0;
    return MF4D_OK;
}

int mf4d_grow_batched(mf4d_ctx* c, uint32_t* fplanes, size_t fwords, uint32_t* pplanes,
                      size_t pwords, int where, mf4d_stats* out) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (!c->has_field) return fail(MF4D_ERR_STATE, "no field loaded");
    if (c->Q == 0) return fail(MF4D_ERR_STATE, "no queries set");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    const Geom& g = c->g;
    const uint64_t V = (uint64_t)g.X * g.Y * g.Z * g.T;
    const uint64_t P = c->has_particles ? (uint64_t)c->pg.P : 0;
    const uint64_t Tp = P > 0 ? (uint64_t)c->pg.T : 0;
    // no buffers: grow into planes the context owns (read with mf4d_read_batched)
    const bool owned = !fplanes && !pplanes && fwords == 0 && pwords == 0;
    if (!owned) {
        if (!fplanes || fwords < 8 * V)
            return fail(MF4D_ERR_ARG, "field planes need %llu words", (unsigned long long)(8 * V));
        if (P > 0 && (!pplanes || pwords < 8 * P * Tp))
            return fail(MF4D_ERR_ARG, "particle planes need %llu words", (unsigned long long)(8 * P * Tp));
        if ((reinterpret_cast<uintptr_t>(fplanes) & 15) || (reinterpret_cast<uintptr_t>(pplanes) & 15))
            return fail(MF4D_ERR_ARG, "plane buffers must be 16-byte aligned");
    }
    HIP_TRY(hipSetDevice(c->device));
    c->b_grown = false;
    if (owned) {
        if (c->b_fown_n < 8 * V) {
            dev_free(c->b_fown);
            c->b_fown_n = 0;
            int rc = dev_alloc(&c->b_fown, (size_t)(8 * V));
            if (rc) return rc;
            c->b_fown_n = (size_t)(8 * V);
        }
        if (P > 0 && c->b_pown_n < 8 * P * Tp) {
            dev_free(c->b_pown);
            c->b_pown_n = 0;
            int rc = dev_alloc(&c->b_pown, (size_t)(8 * P * Tp));
            if (rc) return rc;
            c->b_pown_n = (size_t)(8 * P * Tp);
        }
        fplanes = c->b_fown;
        pplanes = P > 0 ? c->b_pown : nullptr;
        where = MF4D_DEVICE;
    }
    if (c->NTB == 0) {
        const int NXb = (g.X + (1 << c->blog[0]) - 1) >> c->blog[0];
        const int NYb = (g.Y + (1 << c->blog[1]) - 1) >> c->blog[1];
        const int NZb = (g.Z + (1 << c->blog[2]) - 1) >> c->blog[2];
        const int NTb = (g.T + (1 << c->blog[3]) - 1) >> c->blog[3];
        const uint64_t ntb = (uint64_t)NXb * NYb * NZb * NTb;
        int rc = dev_alloc(&c->b_active, (size_t)ntb + 8);
        if (!rc) rc = dev_alloc(&c->b_dirty, 2 * (size_t)ntb);
        if (!rc) rc = dev_alloc(&c->b_chg, 2 * (size_t)ntb + 8);
        const uint32_t wcap = (uint32_t)((ntb + kBSubs - 1) / kBSubs);
        if (!rc) rc = dev_alloc(&c->b_work, 2 * (size_t)kBSubs * wcap);
        if (!rc && !c->b_wcnt) rc = dev_alloc(&c->b_wcnt, 2 * (size_t)kBSubs * kBCntStride);
        if (!rc && !c->b_counters) rc = dev_alloc(&c->b_counters, BC_NCOUNTERS);
        if (rc) {
            dev_free(c->b_active);
            dev_free(c->b_dirty);
            dev_free(c->b_chg);
            dev_free(c->b_work);
            dev_free(c->b_wcnt);
            return rc;
        }
        c->b_wcap = wcap;
        c->NXb = NXb; c->NYb = NYb; c->NZb = NZb; c->NTb = NTb;
        c->NTB = (uint32_t)ntb;
    }
    if (!c->b_vrank) {
        int rc = dev_alloc(&c->b_vrank, (size_t)V);
        if (rc) return rc;
    }
    if (P > 0 && !c->b_prank) {
        int rc = dev_alloc(&c->b_prank, (size_t)P * c->pg.Tpad);
        if (rc) return rc;
    }
    uint32_t* fo = fplanes;
    uint32_t* po = pplanes;
    if (where == MF4D_HOST) {
        void* st = nullptr;
        int rc = staging_for(c, (size_t)(8 * V + 8 * P * Tp) * sizeof(uint32_t), &st);
        if (rc) return rc;
        fo = (uint32_t*)st;
        po = fo + 8 * V;
    }
    DevB d{};
    d.g = g;
    d.X = g.X; d.Y = g.Y; d.Z = g.Z; d.T = g.T;
    d.Tp = (int)Tp;
    d.NXb = c->NXb; d.NYb = c->NYb; d.NZb = c->NZb; d.NTb = c->NTb;
    d.lx = c->blog[0]; d.ly = c->blog[1]; d.lz = c->blog[2]; d.lt = c->blog[3];
    d.NTB = c->NTB;
    d.Q = c->Q;
    d.P = (int64_t)P;
    d.Tpad = c->has_particles ? c->pg.Tpad : 1;
    d.field = c->field;
    d.attr_t = c->attr_t;
    d.vrank = c->b_vrank;
    d.prank = P > 0 ? c->b_prank : nullptr;
    d.bins = c->bins;
    d.fplanes = fo;
    d.pplanes = P > 0 ? po : nullptr;
    d.tab = c->btab;
    d.active = c->b_active;
    d.dirty = c->b_dirty;
    d.chg = c->b_chg;
    d.work = c->b_work;
    d.wcnt = c->b_wcnt;
    d.WCAPB = c->b_wcap;
    d.clist = c->clist;
    d.pdirty = c->pdirty;
    d.dlist = c->dlist;
    d.counters = c->b_counters;
    d.stat64 = c->stat64;
    d.forward_only = c->forward_only;
    hipStream_t s = c->stream;
    HIP_TRY(hipEventRecord(c->ev[0], s));
    launch_b_prepare(d, c->qseeds, c->QS, s);
    HIP_TRY(hipEventRecord(c->ev[1], s));
    // rounds are queued a chunk at a time (a round with an empty work list is
    // a no-op on the device, and every round after it is one too); the host
    // reads the counters once per chunk
    constexpr uint32_t kChunk = 8;
    uint32_t r = 0;
    while (true) {
        launch_fill_u32(c->b_counters + BC_ROUNDS, 0, 1, s);
        for (uint32_t k = 0; k < kChunk; ++k) launch_b_round(d, r + k, s);
        launch_b_work_total(d, 0, s);
        launch_b_work_total(d, 1, s);
        HIP_TRY(hipMemcpyAsync(c->h_counters, c->b_counters, BC_NCOUNTERS * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s));
        int rc = sync(c);
        if (rc) return rc;
        const uint32_t done = c->h_counters[BC_ROUNDS];
        r += done;
        if (done < kChunk || c->h_counters[BC_NWORK0 + (r & 1)] == 0) break;
    }
    HIP_TRY(hipEventRecord(c->ev[3], s));
    HIP_TRY(hipMemcpyAsync(c->h_stat, c->stat64, S_NSTAT * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    int rc = sync(c);
    if (rc) return rc;
    mf4d_stats st{};
    st.rounds = r;
    st.tile_visits = (int64_t)c->h_stat[S_TILE_VISITS];
    st.particle_visits = (int64_t)c->h_stat[S_PART_VISITS];
    st.seeds_dropped = (int64_t)c->h_counters[BC_DROPPED];
    st.members_field = -1;
    st.members_particle = -1;
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    st.ms_admit = ms;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[1], c->ev[3]));
    st.ms_rounds = ms;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[3]));
    st.ms_total = ms;
    if (where == MF4D_HOST) {
        HIP_TRY(hipMemcpyAsync(fplanes, fo, 8 * V * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        if (P > 0)
            HIP_TRY(hipMemcpyAsync(pplanes, po, 8 * P * Tp * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        rc = sync(c);
        if (rc) return rc;
    }
    c->b_grown = owned;
    if (out) *out = st;
    return MF4D_OK;
}

int mf4d_read_batched(mf4d_ctx* c, uint32_t* fdst, size_t fwords, uint32_t* pdst, size_t pwords,
                      int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (!c->b_grown) return fail(MF4D_ERR_STATE, "no batched grow into the context's planes");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    const Geom& g = c->g;
    const uint64_t V = (uint64_t)g.X * g.Y * g.Z * g.T;
    const uint64_t P = c->has_particles ? (uint64_t)c->pg.P : 0;
    const uint64_t Tp = P > 0 ? (uint64_t)c->pg.T : 0;
    if (!fdst || fwords < 8 * V) return fail(MF4D_ERR_ARG, "field planes need %llu words", (unsigned long long)(8 * V));
    if (pdst && pwords < 8 * P * Tp)
        return fail(MF4D_ERR_ARG, "particle planes need %llu words", (unsigned long long)(8 * P * Tp));
    HIP_TRY(hipSetDevice(c->device));
    const hipMemcpyKind k = where == MF4D_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    HIP_TRY(hipMemcpyAsync(fdst, c->b_fown, 8 * V * sizeof(uint32_t), k, c->stream));
    if (pdst && P > 0) HIP_TRY(hipMemcpyAsync(pdst, c->b_pown, 8 * P * Tp * sizeof(uint32_t), k, c->stream));
    return sync(c);
}

int mf4d_set_predictor(mf4d_ctx* c, mf4d_net* net, float logit_threshold) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    settle_submit(c);  // a submitted grow first
    if (logit_threshold != logit_threshold) return fail(MF4D_ERR_ARG, "threshold is NaN");
    c->net = net;
    c->pred_thr = logit_threshold;
    return MF4D_OK;
}

int mf4d_set_scheduler(mf4d_ctx* c, int kind, const void* params, size_t nbytes) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    settle_submit(c);  // a submitted grow first
    if (kind == MF4D_SCHEDULER_PLAIN || kind == MF4D_SCHEDULER_HEURISTIC) {
        if (params || nbytes) return fail(MF4D_ERR_ARG, "this scheduler takes no parameters");
        c->net = nullptr;
        c->pred_thr = 0.0f;
        c->priority = kind;
        return MF4D_OK;
    }
    if (kind != MF4D_SCHEDULER_LEARNED) return fail(MF4D_ERR_ARG, "unknown scheduler %d", kind);
    const int np = mf4d_net_num_params();
    if (!params || nbytes != (size_t)(np + 1) * sizeof(float))
        return fail(MF4D_ERR_ARG, "the learned scheduler takes %d fp32 parameters and a threshold", np);
    const float thr = static_cast<const float*>(params)[np];
    if (thr != thr) return fail(MF4D_ERR_ARG, "threshold is NaN");
    if (!c->own_net) {
        int rc = mf4d_net_create(&c->own_net, c->device, c->stream);
        if (rc) return fail(rc, "network: %s", mf4d_net_last_error());
    }
    int rc = mf4d_net_set_params(c->own_net, static_cast<const float*>(params), MF4D_HOST);
    if (rc) return fail(rc, "network: %s", mf4d_net_last_error());
    c->net = c->own_net;
    c->pred_thr = thr;
    c->priority = MF4D_SCHEDULER_LEARNED;
    return MF4D_OK;
}

int mf4d_features(mf4d_ctx* c, uint16_t* dst, size_t n, int where) {
    if (!c || !dst) return fail(MF4D_ERR_ARG, "NULL argument");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (!c->has_field || !c->has_crit) return fail(MF4D_ERR_STATE, "load a field and set criteria first");
    const size_t need = (size_t)c->bd.T * c->bd.D * c->bd.H * c->bd.W * 16;
    if (n < need) return fail(MF4D_ERR_ARG, "dst holds %zu elements, %zu needed", n, need);
    HIP_TRY(hipSetDevice(c->device));
    ensure_brick_stats(c);
    launch_features(c->bd, c->bstats, c->crit[0], c->feat, c->stream);
    HIP_TRY(hipMemcpyAsync(dst, c->feat, need * sizeof(uint16_t),
                           where == MF4D_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                           c->stream));
    return sync(c);
}

int mf4d_brick_labels(mf4d_ctx* c, uint8_t* dst, size_t n, int where) {
    if (!c || !dst) return fail(MF4D_ERR_ARG, "NULL argument");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (c->state == 0) return fail(MF4D_ERR_STATE, "nothing grown");
    const size_t need = (size_t)c->bd.T * c->bd.D * c->bd.H * c->bd.W;
    if (n < need) return fail(MF4D_ERR_ARG, "dst holds %zu bytes, %zu needed", n, need);
    HIP_TRY(hipSetDevice(c->device));
    uint8_t* out = dst;
    if (where == MF4D_HOST) {
        void* st = nullptr;
        int rc = staging_for(c, need, &st);
        if (rc) return rc;
        out = (uint8_t*)st;
    }
    launch_brick_labels(c->g, c->bd, c->Lf, c->active, out, c->stream);
    if (where == MF4D_HOST)
        HIP_TRY(hipMemcpyAsync(dst, out, need, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int mf4d_brick_dims(mf4d_ctx* c, int* dims4) {
    if (!c || !dims4) return fail(MF4D_ERR_ARG, "NULL argument");
    if (!c->has_field) return fail(MF4D_ERR_STATE, "no field loaded");
    dims4[0] = c->bd.T;
    dims4[1] = c->bd.D;
    dims4[2] = c->bd.H;
    dims4[3] = c->bd.W;
    return MF4D_OK;
}

int mf4d_last_stats(mf4d_ctx* c, mf4d_stats* out) {
    if (!c || !out) return fail(MF4D_ERR_ARG, "NULL argument");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (c->state == 0) return fail(MF4D_ERR_STATE, "nothing grown");
    int rc = settle_members(c);
    if (rc) return rc;
    *out = c->stats;
    return MF4D_OK;
}

// ---------------------------------------------------------------------------
// 4D SLIC clustering (Section 3.2)

int mf4d_slic_set_params(mf4d_ctx* c, const int* k4, float w_d, float w_f, float w_p, float c_f,
                         double eps, int max_iter) {
    if (!c || !k4) return fail(MF4D_ERR_ARG, "NULL argument");
    settle_submit(c);  // a submitted grow first
    int64_t K = 1;
    for (int i = 0; i < 4; ++i) {
        if (k4[i] < 1 || k4[i] > 4096) return fail(MF4D_ERR_ARG, "k[%d] = %d not in [1, 4096]", i, k4[i]);
        K *= k4[i];
    }
    if (K > (1 << 24)) return fail(MF4D_ERR_ARG, "%lld centres exceed 2^24", (long long)K);
    const float w[4] = {w_d, w_f, w_p, c_f};
    for (int i = 0; i < 4; ++i)
        if (!(w[i] >= 0.0f && w[i] <= 3.4e38f)) return fail(MF4D_ERR_ARG, "weights and c_f must be finite and >= 0");
    if (!(eps >= 0.0 && eps <= 1.7e308)) return fail(MF4D_ERR_ARG, "eps must be finite and >= 0");
    if (max_iter < 0 || max_iter > 100000) return fail(MF4D_ERR_ARG, "max_iter %d not in [0, 100000]", max_iter);
    HIP_TRY(hipSetDevice(c->device));
    if ((int)K != c->sK) {
        dev_free(c->sacc);
        dev_free(c->scen);
        dev_free(c->scen32);
        dev_free(c->scnt);
        dev_free(c->slsum);
        dev_free(c->mbuf);
        c->merged = false;
        c->sK = 0;
        int rc = dev_alloc(&c->sacc, (size_t)K * kSlicAcc);
        if (!rc) rc = dev_alloc(&c->scen, (size_t)K * 6);
        if (!rc) rc = dev_alloc(&c->scen32, (size_t)K * 8);
        if (!rc) rc = dev_alloc(&c->scnt, (size_t)K * 2);
        if (!rc) rc = dev_alloc(&c->slsum, (size_t)K * kSlicAcc);
        if (!rc && !c->scounters) rc = dev_alloc(&c->scounters, (size_t)kSlicCounters);
        if (!rc && !c->sslab) rc = dev_alloc(&c->sslab, (size_t)16 * 4096);
        if (!rc && !c->h_scounters &&
            hipHostMalloc((void**)&c->h_scounters, kSlicCounters * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
            rc = fail(MF4D_ERR_OOM, "pinned counters");
        if (rc) return rc;
        c->sK = (int)K;
    }
    for (int i = 0; i < 4; ++i) c->sk[i] = k4[i];
    c->swd = w_d;
    c->swf = w_f;
    c->swp = w_p;
    c->scf = c_f;
    c->seps = eps;
    c->smax_iter = max_iter;
    c->slic_params = true;
    c->slic_done = false;
    return MF4D_OK;
}

int mf4d_slic_run(mf4d_ctx* c, int* iterations) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    {
        const int rs = settle_async(c);  // asynchronous read-outs still running
        if (rs) return rs;
    }
    if (!c->has_field) return fail(MF4D_ERR_STATE, "no field loaded");
    if (!c->slic_params) return fail(MF4D_ERR_STATE, "no clustering parameters set");
    const Geom& g = c->g;
    if (g.X >= 2048 || g.Y >= 2048 || g.Z >= 2048 || g.T >= 2048)
        return fail(MF4D_ERR_UNSUPPORTED, "clustering needs every dimension below 2048");
    const int64_t P = c->has_particles ? c->pg.P : 0;
    const size_t V = (size_t)g.X * g.Y * g.Z * g.T, Qp = P > 0 ? (size_t)c->pg.T * P : 0;
    if (V + Qp >= (size_t)1 << 31) return fail(MF4D_ERR_UNSUPPORTED, "more than 2^31 samples");
    HIP_TRY(hipSetDevice(c->device));
    c->slic_done = false;
    if (c->slabels_n != V + Qp) {
        dev_free(c->slabels);
        c->slabels_n = 0;
        int rc = dev_alloc(&c->slabels, V + Qp);
        if (rc) return rc;
        c->slabels_n = V + Qp;
    }
    if (P > 0 && !c->porder) {
        // point samples in tile order, so that a block of them meets few centres
        int rc = dev_alloc(&c->porder, Qp);
        if (!rc) rc = dev_alloc(&c->spos, Qp);
        if (!rc) rc = dev_alloc(&c->sattr, Qp);
        uint32_t* scratch = nullptr;
        if (!rc) rc = dev_alloc(&scratch, (size_t)g.NT + 1 + 1 + 1025);
        if (!rc) {
            const int e = launch_slic_order(c->bins, c->praw, c->praw + (size_t)3 * Qp, P, c->pg.Tpad, c->pg.T,
                                            c->pg.tr, 5 + 6 + g.logBT, g.NT, scratch, c->porder, c->spos,
                                            c->sattr, c->stream);
            if (e != hipSuccess) rc = fail(MF4D_ERR_HIP, "clustering order: %s", hipGetErrorString((hipError_t)e));
        }
        if (!rc) rc = sync(c);
        dev_free(scratch);
        if (rc) {
            dev_free(c->porder);
            dev_free(c->spos);
            dev_free(c->sattr);
            return rc;
        }
    }
    DevS s{};
    s.X = g.X; s.Y = g.Y; s.Z = g.Z; s.T = g.T;
    s.P = P;
    s.Tp = P > 0 ? c->pg.T : 0;
    for (int i = 0; i < 4; ++i) s.k[i] = c->sk[i];
    s.K = c->sK;
    const float E[4] = {(float)g.X, (float)g.Y, (float)g.Z, (float)g.T};
    for (int i = 0; i < 4; ++i) s.C[i] = E[i] / (float)c->sk[i];
    s.wd = c->swd; s.wf = c->swf; s.wp = c->swp; s.cf = c->scf;
    s.eps = c->seps;
    s.field = c->field;
    s.spos = P ? c->spos : nullptr;
    s.sattr = P ? c->sattr : nullptr;
    s.labels = c->slabels;
    s.acc = c->sacc;
    s.cen = c->scen;
    s.cen32 = c->scen32;
    s.cnt = c->scnt;
    s.counters = c->scounters;
    s.slab = c->sslab;
    s.reach = reinterpret_cast<int*>(c->sslab + 8 * 4096);
    // debug switch: MF4D_SLIC_MASK_SLABS = 0 sends every sample through the
    // general candidate loop (the tests compare both paths)
    s.mask_slabs = 32;
    if (const char* e = getenv("MF4D_SLIC_MASK_SLABS")) s.mask_slabs = std::min(32, std::max(0, atoi(e)));
    s.lsum = c->slsum;
    s.kmax = std::max(std::max(c->sk[0], c->sk[1]), std::max(c->sk[2], c->sk[3]));
    hipStream_t st = c->stream;
    launch_fill_u32((uint32_t*)c->sacc, 0, (uint64_t)c->sK * kSlicAcc * 2, st);
    launch_fill_u32(c->scounters, 0, kSlicCounters, st);
    launch_slic_init(s, st);
    launch_slic_update(s, 1, st);
    int it = 0;
    while (it < c->smax_iter) {
        launch_fill_u32(c->scounters + SC_MOVED, 0, 1, st);
        launch_slic_assign(s, st);
        ++it;
        launch_slic_update(s, 0, st);
        HIP_TRY(hipMemcpyAsync(c->h_scounters, c->scounters, kSlicCounters * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, st));
        int rc = sync(c);
        if (rc) return rc;
        if (c->h_scounters[SC_RANGE]) break;
        if (c->h_scounters[SC_MOVED] == 0) break;
    }
    HIP_TRY(hipMemcpyAsync(c->h_scounters, c->scounters, kSlicCounters * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, st));
    int rc = sync(c);
    if (rc) return rc;
    if (c->h_scounters[SC_RANGE])
        return fail(MF4D_ERR_RANGE, "a coordinate or value with |v| >= 2048: the clustering's exact sums could overflow");
    c->slic_iters = it;
    c->slic_done = true;
    c->merged = false;
    if (iterations) *iterations = it;
    return MF4D_OK;
}

int mf4d_slic_read_labels(mf4d_ctx* c, int32_t* field_labels, size_t nf, int32_t* point_labels, size_t np,
                          int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->slic_done) return fail(MF4D_ERR_STATE, "no clustering run");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    const Geom& g = c->g;
    const size_t V = (size_t)g.X * g.Y * g.Z * g.T, Qp = c->slabels_n - V;
    if (field_labels && nf < V) return fail(MF4D_ERR_ARG, "field labels hold %zu, %zu needed", nf, V);
    if (point_labels && np < Qp) return fail(MF4D_ERR_ARG, "point labels hold %zu, %zu needed", np, Qp);
    HIP_TRY(hipSetDevice(c->device));
    const hipMemcpyKind kind = where == MF4D_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (field_labels) HIP_TRY(hipMemcpyAsync(field_labels, c->slabels, V * sizeof(int32_t), kind, c->stream));
    if (point_labels && Qp) {
        // point labels are kept in visiting order: put them back in [T][P]
        int32_t* out = point_labels;
        if (where == MF4D_HOST) {
            void* st = nullptr;
            int rc = staging_for(c, Qp * sizeof(int32_t), &st);
            if (rc) return rc;
            out = (int32_t*)st;
        }
        launch_slic_unsort(c->slabels + V, c->porder, Qp, out, c->stream);
        if (where == MF4D_HOST)
            HIP_TRY(hipMemcpyAsync(point_labels, out, Qp * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    }
    if (where == MF4D_DEVICE) return MF4D_OK;  // stream-ordered
    return sync(c);
}

int mf4d_slic_read_centres(mf4d_ctx* c, double* centres, int64_t* counts, size_t K, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->slic_done) return fail(MF4D_ERR_STATE, "no clustering run");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    if (K < (size_t)c->sK) return fail(MF4D_ERR_ARG, "room for %zu centres, %d needed", K, c->sK);
    HIP_TRY(hipSetDevice(c->device));
    const hipMemcpyKind kind = where == MF4D_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (centres) HIP_TRY(hipMemcpyAsync(centres, c->scen, (size_t)c->sK * 6 * sizeof(double), kind, c->stream));
    if (counts) HIP_TRY(hipMemcpyAsync(counts, c->scnt, (size_t)c->sK * 2 * sizeof(int64_t), kind, c->stream));
    if (where == MF4D_DEVICE) return MF4D_OK;  // stream-ordered
    return sync(c);
}

// The clustering's device state for the merge (the last run's buffers).
static DevS slic_state(mf4d_ctx* c) {
    const Geom& g = c->g;
    DevS s{};
    s.X = g.X; s.Y = g.Y; s.Z = g.Z; s.T = g.T;
    s.P = c->has_particles ? c->pg.P : 0;
    s.Tp = s.P > 0 ? c->pg.T : 0;
    for (int i = 0; i < 4; ++i) s.k[i] = c->sk[i];
    s.K = c->sK;
    s.field = c->field;
    s.spos = s.P ? c->spos : nullptr;
    s.sattr = s.P ? c->sattr : nullptr;
    s.labels = c->slabels;
    s.cen = c->scen;
    s.cnt = c->scnt;
    s.lsum = c->slsum;
    return s;
}

int mf4d_slic_merge(mf4d_ctx* c, double eps_m, int* n_features) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->slic_done) return fail(MF4D_ERR_STATE, "no clustering run");
    if (!(eps_m >= 0.0 && eps_m <= 1.7e308)) return fail(MF4D_ERR_ARG, "eps_m must be finite and >= 0");
    HIP_TRY(hipSetDevice(c->device));
    const size_t K = (size_t)c->sK;
    if (!c->mbuf) {
        // parent, feat (int), fsum (8 x u64), fmean (2 x f64), cext, fext (8 x u32),
        // css, fss (2 x f64), out (kFeatStats x f64), err
        // ten arrays, each started on a 256-byte boundary
        const size_t bytes = K * (4 + 4 + 64 + 16 + 32 + 32 + 16 + 16 + 8 * kFeatStats) + 10 * 256;
        int rc = dev_alloc(&c->mbuf, bytes);
        if (rc) return rc;
        char* p = c->mbuf;
        auto take = [&](size_t n) { char* q = p; p += (n + 255) / 256 * 256; return q; };
        DevM& m = c->m;
        m.K = (int)K;
        m.fsum = (unsigned long long*)take(K * 64);
        m.fmean = (double*)take(K * 16);
        m.css = (double*)take(K * 16);
        m.fss = (double*)take(K * 16);
        m.out = (double*)take(K * 8 * kFeatStats);
        m.cext = (uint32_t*)take(K * 32);
        m.fext = (uint32_t*)take(K * 32);
        m.parent = (int*)take(K * 4);
        m.feat = (int32_t*)take(K * 4);
        m.err = (uint32_t*)take(4);
        if ((size_t)(p - c->mbuf) > bytes) {
            dev_free(c->mbuf);
            return fail(MF4D_ERR_HIP, "internal error: merge buffer layout");
        }
    }
    c->m.eps = eps_m;
    launch_fill_u32(c->m.err, 0, 1, c->stream);
    const int e = launch_slic_merge(slic_state(c), c->m, c->stream);
    if (e != hipSuccess) return fail(MF4D_ERR_HIP, "merge: %s", hipGetErrorString((hipError_t)e));
    std::vector<int32_t> feat(K);
    uint32_t err = 0;
    HIP_TRY(hipMemcpyAsync(feat.data(), c->m.feat, K * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(&err, c->m.err, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    int rc = sync(c);
    if (rc) return rc;
    if (err) return fail(MF4D_ERR_HIP, "internal error: a union-find walk did not end");
    int n = 0;
    for (size_t i = 0; i < K; ++i) n += feat[i] == (int32_t)i;
    if (n_features) *n_features = n;
    c->merged = true;
    return MF4D_OK;
}

int mf4d_slic_read_features(mf4d_ctx* c, int32_t* feature_of_centre, double* stats, size_t K, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->slic_done || !c->merged) return fail(MF4D_ERR_STATE, "no merge since the last clustering run");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    if (K < (size_t)c->sK) return fail(MF4D_ERR_ARG, "room for %zu centres, %d needed", K, c->sK);
    HIP_TRY(hipSetDevice(c->device));
    const hipMemcpyKind kind = where == MF4D_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (feature_of_centre)
        HIP_TRY(hipMemcpyAsync(feature_of_centre, c->m.feat, (size_t)c->sK * sizeof(int32_t), kind, c->stream));
    if (stats)
        HIP_TRY(hipMemcpyAsync(stats, c->m.out, (size_t)c->sK * kFeatStats * sizeof(double), kind, c->stream));
    if (where == MF4D_DEVICE) return MF4D_OK;  // stream-ordered
    return sync(c);
}

int mf4d_slic_read_segments(mf4d_ctx* c, int32_t* dst, size_t n, int where) {
    if (!c) return fail(MF4D_ERR_ARG, "ctx is NULL");
    if (!c->slic_done || !c->merged) return fail(MF4D_ERR_STATE, "no merge since the last clustering run");
    if (!dst) return fail(MF4D_ERR_ARG, "dst is NULL");
    if (where != MF4D_HOST && where != MF4D_DEVICE) return fail(MF4D_ERR_ARG, "bad where");
    const Geom& g = c->g;
    const size_t V = (size_t)g.X * g.Y * g.Z * g.T, Qp = c->slabels_n - V;
    if (Qp == 0) return fail(MF4D_ERR_STATE, "the last clustering run had no point samples");
    if (n < Qp) return fail(MF4D_ERR_ARG, "dst holds %zu, %zu needed", n, Qp);
    HIP_TRY(hipSetDevice(c->device));
    int32_t* out = dst;
    if (where == MF4D_HOST) {
        void* st = nullptr;
        int rc = staging_for(c, Qp * sizeof(int32_t), &st);
        if (rc) return rc;
        out = (int32_t*)st;
    }
    launch_slic_unsort(c->slabels + V, c->porder, Qp, out, c->stream);
    launch_slic_segments(out, c->m.feat, c->pg.T, (int64_t)(Qp / c->pg.T), c->stream);
    if (where == MF4D_HOST)
        HIP_TRY(hipMemcpyAsync(dst, out, Qp * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    if (where == MF4D_DEVICE) return MF4D_OK;  // stream-ordered
    return sync(c);
}

}  // extern "C"
