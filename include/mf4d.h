/*
 * mf4d -- coupled point + field 4D region growing on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libmf4d.so.  Plain pointers and sizes only.
 *
 * The data model follows Sauer & Ma, "Multifaceted 4D Feature Segmentation
 * and Extraction in Point and Field-based Datasets", Section 3.1: field
 * samples F(t) = {x_f, y_f, z_f, v_f(t)} on a fixed regular grid and point
 * samples P(t) = {x_p(t), y_p(t), z_p(t), v_p(t)} that move and form
 * trajectories.  The grown feature has a field part and a point part and
 * spans timesteps (Section 1, contributions).
 *
 * Operation.  Nodes are voxel-steps (x, y, z, t) and particle-steps (i, t).
 * A voxel-step is admissible iff f_lo <= f <= f_hi and a particle-step iff
 * a_lo <= a <= a_hi, compared in fp32 on the stored values; NaN is never
 * admissible.  (Each sample type is tested only on its own value, as the
 * paper's D_f and D_p compare each sample type only with its own variable,
 * Section 3.2.3.)  Undirected edges join a voxel to its six spatial face
 * neighbours and to the same voxel at t-1 and t+1 (no wrap-around); a
 * particle-step to the voxel whose volume holds it (the field-to-point index
 * of Section 3.1; voxel i covers [i, i+1) per axis in voxel units, and a
 * position outside [0, dim) or NaN lies in no voxel); and a particle-step to
 * the same particle at t-1 and t+1 (trajectories connect points between
 * timesteps, Section 1).  The grown set is every node reachable from the
 * admissible seeds through admissible nodes.  Seeds that are not admissible
 * are dropped and counted.
 *
 * Layouts.
 *   field      fp32 [T][Z][Y][X]
 *   xyz        fp32 [T][P][3], positions already in voxel units
 *   attr       fp32 [T][P]
 *   seeds      int32 [S][4] = (x, y, z, t)
 *   field mask uint32 words: voxel-step bit ((t*Z + z)*Y + y)*X + x lives in
 *              word bit >> 5 at bit position bit & 31; bits past the end of
 *              the grid in the last word are zero
 *   particle mask uint8 [T][P], 1 = member
 *
 * Ownership and streams.  A context owns every device buffer it allocates.
 * Caller pointers are borrowed for the duration of a call only; each pointer
 * argument is accompanied by `where` (MF4D_HOST or MF4D_DEVICE).  All work is
 * ordered on the HIP stream given at creation (NULL = the null stream).
 * Load and read calls return once their copies are complete; mf4d_grow
 * returns once the grown set is complete on the device.
 *
 * Errors.  Every call returns MF4D_OK or a negative status and records a
 * message readable with mf4d_last_error() (per thread).  Arguments are
 * validated before any state changes, so a failed call leaves the context as
 * it was (except MF4D_ERR_HIP, after which the context should be destroyed).
 * No C++ exception crosses this interface.
 */
#ifndef MF4D_H
#define MF4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mf4d_ctx mf4d_ctx;
typedef struct mf4d_net mf4d_net;

enum {
    MF4D_OK = 0,
    MF4D_ERR_ARG = -1,           /* bad pointer, size or value */
    MF4D_ERR_RANGE = -2,         /* a seed outside the grid */
    MF4D_ERR_OOM = -3,           /* device allocation failed */
    MF4D_ERR_HIP = -4,           /* a HIP runtime call failed */
    MF4D_ERR_STATE = -5,         /* call out of order (e.g. grow before load) */
    MF4D_ERR_NOT_CONVERGED = -6, /* round cap reached; masks hold a valid subset */
    MF4D_ERR_UNSUPPORTED = -7    /* shape outside what the library supports */
};

enum { MF4D_HOST = 0, MF4D_DEVICE = 1 };

/* Admissibility modes (mf4d_set_admit_mode). */
enum { MF4D_ADMIT_TILES = 0, MF4D_ADMIT_ALL = 1 };

/* Schedulers of the rounds of a grow (mf4d_set_scheduler). */
enum {
    MF4D_SCHEDULER_PLAIN = 0,    /* tiles are visited in the order their work is found */
    MF4D_SCHEDULER_LEARNED = 1,  /* the brick-activity predictor orders the first visits */
    MF4D_SCHEDULER_HEURISTIC = 2 /* the tiles' greatest field values order the first visits */
};

/* Trajectory coupling (mf4d_set_trajectory_mode). */
enum { MF4D_TRAJ_BOTH = 0, MF4D_TRAJ_FORWARD = 1 };

/* How the rounds of a grow are scheduled (both give the same result). */
enum {
    MF4D_SCHED_PERSISTENT = 0, /* one cooperative kernel runs every round (default) */
    MF4D_SCHED_LAUNCH = 1,     /* three kernel launches per round */
    MF4D_SCHED_JACOBI = 2      /* debugging: synchronous sweeps over every node, one edge per sweep;
                                  converges after D + 1 sweeps, D the largest breadth-first level
                                  (stats.rounds counts the sweeps; admissibility is read everywhere) */
};

typedef struct mf4d_stats {
    int64_t rounds;           /* rounds run: each sweeps its work list, pulls, closes and pushes;
                                 the grow stops when the next round's work list is empty */
    int64_t tile_visits;      /* tile sweeps executed over all rounds */
    int64_t particle_visits;  /* particle closures executed over all rounds */
    int64_t members_field;    /* |M ∩ voxel-steps| (filled by mf4d_read_field_mask) */
    int64_t members_particle; /* |M ∩ particle-steps| (filled by mf4d_read_particle_mask) */
    int64_t seeds_dropped;    /* seed entries that failed the field criterion */
    int64_t active_tiles;     /* tiles holding at least one admissible voxel-step */
    double ms_admit_field;    /* admissibility pass over the field (one kernel) */
    double ms_admit;          /* admissibility pass over field and particles */
    double ms_rounds;         /* seeding and all rounds */
    double ms_total;          /* the whole mf4d_grow call on the device */
    int64_t tiles_tested;     /* single-query grow: tiles whose admissibility was read before the rounds
                                 (every tile when admissibility is tested everywhere) */
    int64_t tiles_deferred_read; /* deferred tiles whose admissibility a sweep read */
    double ms_sweep;          /* rounds as launches: device time of the sweep kernels (summed over
                                 the rounds that had work; 0 for the persistent schedule) */
    double ms_pull;           /* likewise for the pull kernels */
    double ms_close;          /* likewise for the close/push kernels */
    int64_t coupled_steps;    /* single-query grow: admissible particle-steps that lie in a voxel */
    int64_t priority_visits;  /* score-ordered schedulers: tiles swept by the priority pass */
    int64_t verify_rounds;    /* score-ordered schedulers: rounds from the verification round on
                                 (1 when it changed nothing); included in `rounds` */
} mf4d_stats;

/* Record HIP events in each grow (on = 1) so that the device times of
 * mf4d_stats (ms_admit_field, ms_admit, ms_rounds, ms_total, and for rounds
 * run as launches ms_sweep / ms_pull / ms_close) are filled; off (0, the
 * default) records none and those times read 0: each event costs a few
 * microseconds of device time.  Errors: MF4D_ERR_ARG. */
int mf4d_set_phase_timing(mf4d_ctx *ctx, int on);

/* Library version string. */
const char *mf4d_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *mf4d_last_error(void);

/* Bytes of device memory the grower contexts hold (all devices; networks
 * are not counted).  An environment variable MF4D_MAX_DEVICE_BYTES (decimal),
 * read at each allocation, caps it: an allocation that would exceed the cap
 * fails with MF4D_ERR_OOM as if the device were full (a way to exercise
 * out-of-memory handling); the failing call frees what it allocated. */
int64_t mf4d_device_bytes(void);

/* Create a context on HIP device `device`, ordering its work on `hip_stream`
 * (a hipStream_t, or NULL for the null stream).  *out receives the context.
 * Errors: MF4D_ERR_ARG (out NULL, bad device), MF4D_ERR_HIP. */
int mf4d_create(mf4d_ctx **out, int device, void *hip_stream);

/* Release every device buffer of the context.  NULL is accepted. */
void mf4d_destroy(mf4d_ctx *ctx);

/* Tile shape used for the bit-packed labels: 32 (x, one word) x 8 (y) x 8 (z)
 * x bt (t) voxel-steps, bt in {4, 8, 16}.  Must be called before
 * mf4d_load_field; the default is bt = 8.
 * Errors: MF4D_ERR_ARG (other values), MF4D_ERR_STATE (field already loaded). */
int mf4d_set_tile(mf4d_ctx *ctx, int bt);

/* Load the field samples F(t) (Section 3.1): fp32 [T][Z][Y][X].  Replaces any
 * earlier field and drops loaded particles (they are binned against this
 * grid).  Requires X*Y*Z*T (padded to whole tiles) < 2^32.
 * Errors: MF4D_ERR_ARG, MF4D_ERR_UNSUPPORTED (too large), MF4D_ERR_OOM. */
int mf4d_load_field(mf4d_ctx *ctx, const float *field, int X, int Y, int Z, int T, int where);

/* Load the point samples P(t) (Section 3.1): positions xyz fp32 [T][P][3] in
 * voxel units and values attr fp32 [T][P], with the same T as the field.
 * Bins every particle-step into the voxel covering it (the field-to-point
 * index of Section 3.1).  P = 0 clears the particles.
 * Errors: MF4D_ERR_STATE (no field), MF4D_ERR_ARG (T differs, bad sizes),
 * MF4D_ERR_UNSUPPORTED (P*T padded >= 2^31), MF4D_ERR_OOM. */
int mf4d_load_particles(mf4d_ctx *ctx, const float *xyz, const float *attr, int64_t P, int T,
                        int where);

/* Load point samples stored at their own temporal rate (Section 3.4: point
 * and field data need not share a temporal resolution; particles are often
 * saved more frequently than the field): positions xyz fp32 [Tp][P][3] and
 * values attr fp32 [Tp][P], with r = steps_per_field_step particle steps per
 * field step (1 <= r <= 1024, 1 <= Tp <= r * T).  Particle step tau lies at
 * time tau / r in field steps: it couples with the voxel covering its
 * position at field step floor(tau / r), the step whose interval [t, t + 1)
 * holds that time, and the clustering gives its point sample the time tau / r
 * (fp32).  Trajectory edges join consecutive particle steps.  Every particle
 * output (masks, segments, ids, point labels, batched planes) is then
 * [Tp][P].  r = 1 with Tp = T is mf4d_load_particles.
 * Errors: as mf4d_load_particles; MF4D_ERR_ARG (r or Tp out of range). */
int mf4d_load_particles_rate(mf4d_ctx *ctx, const float *xyz, const float *attr, int64_t P, int Tp,
                             int steps_per_field_step, int where);

/* Membership criteria: inclusive fp32 bands for field and particle values.
 * The paper's method has no thresholds; its metrics D_f and D_p (Section
 * 3.2.3) test each sample type only against its own value, and these bands
 * are that per-type value test made a membership criterion: a voxel-step
 * tests the field band, a particle-step the attribute band.
 * Errors: MF4D_ERR_ARG (a NaN bound). */
int mf4d_set_criteria(mf4d_ctx *ctx, float f_lo, float f_hi, float a_lo, float a_hi);

/* Seeds int32 [S][4] = (x, y, z, t): the field samples (Section 3.1) the
 * grown feature starts from (the paper's method starts from a seed grid of
 * cluster centres, Section 3.2.1; a grower starts from chosen samples
 * instead).  Duplicates are allowed.
 * Errors: MF4D_ERR_STATE (no field), MF4D_ERR_RANGE (a seed outside the
 * grid; nothing changes), MF4D_ERR_ARG. */
int mf4d_set_seeds(mf4d_ctx *ctx, const int32_t *xyzt, int64_t S, int where);

/* Round scheduling, MF4D_SCHED_PERSISTENT or MF4D_SCHED_LAUNCH.  The
 * environment variable MF4D_SCHED=launch selects the latter at creation.  A
 * persistent launch that the device cannot hold co-resident falls back to
 * launches.  Errors: MF4D_ERR_ARG (unknown mode). */
int mf4d_set_schedule(mf4d_ctx *ctx, int mode);

/* Which voxel-steps a grow tests against the field criterion (same result
 * either way).  MF4D_ADMIT_TILES (default): only tiles whose (min, max) field
 * range, summarised once at load, meets the band -- no other tile can hold an
 * admissible voxel.  MF4D_ADMIT_ALL: every voxel-step, one streaming pass.
 * The environment variable MF4D_ADMIT=all selects the latter at creation.
 * Errors: MF4D_ERR_ARG (unknown mode). */
int mf4d_set_admit_mode(mf4d_ctx *ctx, int mode);

/* Direction of the trajectory edges (a particle-step and the same particle
 * at the next step; trajectories carry a feature between timesteps, Section
 * 1).  MF4D_TRAJ_BOTH (default): membership spreads both ways along a run of
 * admissible steps.  MF4D_TRAJ_FORWARD (causal coupling): only from t to
 * t + 1, so a particle joins at the first step that touches the feature and
 * keeps its later admissible steps; the field's t - 1 / t + 1 edges and the
 * particle-voxel coupling stay undirected, and the result is the set that the
 * seeds reach along the directed edges.  Applies to mf4d_grow and
 * mf4d_grow_batched; it invalidates the labels of an earlier grow.
 * Errors: MF4D_ERR_ARG (unknown mode). */
int mf4d_set_trajectory_mode(mf4d_ctx *ctx, int mode);

/* Cap on rounds per mf4d_grow / mf4d_grow_resume call (0 = no cap). */
int mf4d_set_max_rounds(mf4d_ctx *ctx, int64_t cap);

/* Grow the feature from scratch: admissibility of every node, seeding, and
 * rounds of tile sweeps and particle coupling until a round changes no bit.
 * The result is the feature with a field and a point part spanning
 * timesteps of Section 1; every sample is tested independently in each
 * round, as the samples of Section 3.4's GPU design are.
 * `out` (nullable) receives statistics.
 * Errors: MF4D_ERR_STATE (no field or no criteria), MF4D_ERR_NOT_CONVERGED
 * (the round cap was reached: the labels hold a subset of the feature that
 * is reachable from the seeds; mf4d_grow_resume continues), MF4D_ERR_HIP. */
int mf4d_grow(mf4d_ctx *ctx, mf4d_stats *out);

/* Continue rounds from the current labels after MF4D_ERR_NOT_CONVERGED.
 * Errors: as mf4d_grow; MF4D_ERR_STATE if there is nothing to resume. */
int mf4d_grow_resume(mf4d_ctx *ctx, mf4d_stats *out);

/* Discard the grown feature (the output of Section 1's contribution): every
 * field and particle label bit is cleared and the context holds no grown set,
 * so reads fail with MF4D_ERR_STATE and mf4d_grow_resume has nothing to
 * continue until the next mf4d_grow.  (mf4d_grow itself always starts from
 * cleared labels; mf4d_grow_resume is the call that continues from the
 * current ones.)  Waits for the device.
 * Errors: MF4D_ERR_ARG (ctx NULL), MF4D_ERR_STATE (no field loaded). */
int mf4d_reset_labels(mf4d_ctx *ctx);

/* Write the field part of the grown feature as canonical bit words (layout
 * above) to dst, which holds nwords >= ceil(X*Y*Z*T / 32) words.  Counts the
 * members into the statistics of the last grow (see mf4d_last_stats).  With
 * MF4D_DEVICE the call is ordered on the context's stream and returns without
 * waiting for it (dst is ready for later work on that stream); the member
 * count arrives with the stream (mf4d_last_stats waits for it).  With
 * MF4D_HOST it returns when dst is written.
 * Errors: MF4D_ERR_STATE (nothing grown), MF4D_ERR_ARG (dst too small). */
int mf4d_read_field_mask(mf4d_ctx *ctx, uint32_t *dst, size_t nwords, int where);

/* Write the particle part of the grown feature as uint8 [T][P] to dst,
 * which holds n >= T*P bytes.  Stream ordering as mf4d_read_field_mask.
 * Errors: MF4D_ERR_STATE (nothing grown or no particles), MF4D_ERR_ARG. */
int mf4d_read_particle_mask(mf4d_ctx *ctx, uint8_t *dst, size_t n, int where);

/* mf4d_grow followed by mf4d_read_field_mask and mf4d_read_particle_mask
 * into device buffers, in one call: the same labels, masks and statistics.
 * The read-outs are queued on the device behind the rounds, before the host
 * waits to learn that the rounds reached the fixed point, and run only if
 * they did (else they are queued again after the rounds that remain); the
 * particle read-out runs on a second stream beside the field read-out.  With
 * a score-ordered scheduler, Jacobi sweeps or phase timing the read-outs
 * follow the grow as separate calls would.  field_dst (nwords >=
 * ceil(X*Y*Z*T / 32) words) and particle_dst (n >= T*P bytes) are device
 * buffers; either may be NULL to skip that read-out.  Ordered on the
 * context's stream like the MF4D_DEVICE reads: the masks are ready for later
 * work on that stream when the call returns.  On MF4D_ERR_NOT_CONVERGED the
 * masks hold the labels as the round cap left them.
 * Errors: as mf4d_grow; MF4D_ERR_STATE (particle_dst without particles),
 * MF4D_ERR_ARG (a buffer too small). */
int mf4d_grow_read(mf4d_ctx *ctx, uint32_t *field_dst, size_t nwords, uint8_t *particle_dst, size_t n,
                   mf4d_stats *out);

/* Asynchronous read-outs for mf4d_grow_read (on != 0; off by default).  The
 * call returns with its read-outs deferred: the next asynchronous
 * mf4d_grow_read grows on the other of two sets of label words (about
 * X*Y*Z*T / 8 + 9 * T * P bytes more, allocated on first use) and issues
 * them on the library's second stream once its own admissibility passes are
 * queued, so they write the masks beside its rounds.  Every other call on
 * the context (reads, resume, statistics, loads, destroy, ...) and
 * mf4d_read_wait first issue the read-outs still deferred and order the
 * context stream after every read-out still running; until then the caller
 * must not use the masks (synchronising the device is not enough for
 * read-outs not yet issued).  The masks hold the labels as the grow left
 * them, converged or not.  Switching the mode settles the same way.
 * Errors: MF4D_ERR_ARG (ctx NULL). */
int mf4d_set_read_async(mf4d_ctx *ctx, int on);

/* Issue the deferred asynchronous read-outs and order the context stream
 * after every read-out still running (see mf4d_set_read_async); returns
 * without waiting for the device.  Errors: MF4D_ERR_ARG (ctx NULL). */
int mf4d_read_wait(mf4d_ctx *ctx);

/* mf4d_grow_read in two calls, so that the host need not wait for one grow
 * before it queues the next (Section 3.3's iteration to the fixed point,
 * with its end tested later).  mf4d_grow_submit queues the grow (reset,
 * admissibility, seeding, a first chunk of rounds as long as the context's
 * last converged grow, the statistics copy and the read-outs, gated on that
 * chunk reaching the fixed point) and returns without waiting for the
 * device.  mf4d_grow_finish waits for that chunk; if the grow needs more
 * rounds it runs them and the read-outs as mf4d_grow_read would, and it
 * returns the grow's statistics and status (MF4D_ERR_NOT_CONVERGED with a
 * round cap).  Two contexts on two streams, each loaded with the same data,
 * can so keep two grows in flight: one's rounds, bound by the latency of
 * dependent memory accesses, run beside the other's admissibility passes and
 * rounds.  Buffers as mf4d_grow_read; the caller keeps them alive and
 * unused until mf4d_grow_finish has returned and the context stream has
 * reached that point.  Any other call on the context (except
 * mf4d_last_error and mf4d_version) completes a submitted grow first and
 * keeps its result for mf4d_grow_finish.  With a score-ordered scheduler,
 * phase timing, Jacobi sweeps or the persistent schedule, mf4d_grow_submit
 * runs the whole grow at once.
 * Errors (submit): as mf4d_grow_read's argument and state errors;
 * MF4D_ERR_STATE (a submitted grow not yet finished).
 * Errors (finish): MF4D_ERR_STATE (nothing submitted); otherwise the grow's
 * own, as mf4d_grow_read. */
int mf4d_grow_submit(mf4d_ctx *ctx, uint32_t *field_dst, size_t nwords, uint8_t *particle_dst, size_t n);
int mf4d_grow_finish(mf4d_ctx *ctx, mf4d_stats *out);

/* Trajectory segments of the grown feature (Section 3.4, visual
 * representation): a trajectory is split where it leaves the feature, and
 * only pieces of at least two consecutive member steps are kept.  Writes
 * uint8 [T][P] to dst (n >= T*P bytes): 1 where particle p is a member at
 * step t and also at t - 1 or t + 1, else 0.  Reads the labels of the last
 * grow; stream ordering as mf4d_read_particle_mask.
 * Errors: MF4D_ERR_STATE (nothing grown or no particles), MF4D_ERR_ARG. */
int mf4d_read_particle_segments(mf4d_ctx *ctx, uint8_t *dst, size_t n, int where);

/* Per-seed component ids: which seed a grown node belongs to.  Every node gets
 * the index (in the context's seed list) of the lowest seed whose own region
 * -- a grow from that seed alone, with the context's criteria and trajectory
 * mode -- holds it, or -1.  With undirected coupling the regions are the
 * connected components that hold seeds, so each carries its lowest seed; with
 * forward-only coupling regions may overlap and the lowest index wins.  The
 * labelled nodes are exactly those of mf4d_grow.  Runs one grow per seed not
 * already inside an earlier seed's region (*grows, nullable, receives their
 * number), in index order.  field_ids: int32 [T][Z][Y][X], nf >= X*Y*Z*T;
 * particle_ids: int32 [T][P], np >= T*P, or NULL.  Allocates a scratch of
 * 2 bits per voxel-step and 1 bit per particle-step for the call.  Leaves the
 * context with no grown labels (mf4d_grow again before reading masks).
 * Waits for the device.
 * Errors: MF4D_ERR_STATE (no field or no criteria), MF4D_ERR_ARG,
 * MF4D_ERR_NOT_CONVERGED (a round cap stopped a grow), MF4D_ERR_OOM. */
int mf4d_grow_seed_ids(mf4d_ctx *ctx, int32_t *field_ids, size_t nf, int32_t *particle_ids, size_t np,
                       int where, int64_t *grows);

/* Batched queries (up to 256, each with its own criteria and seeds), grown
 * together as the bit-planes of one 256-bit label per node: the interactive
 * loop of the paper's workflow (Section 3: adjust the parameters and segment
 * again) run for many parameter sets in one pass over the data.  crit fp32
 * [Q][4] = (f_lo, f_hi, a_lo, a_hi) per query; seeds int32 [S][5] =
 * (x, y, z, t, q).  Every query means the same as a single grow with its own
 * criteria and seeds.
 * Errors: MF4D_ERR_STATE (no field), MF4D_ERR_ARG (Q not in 1..256, a NaN
 * bound), MF4D_ERR_RANGE (a seed outside the grid or naming q >= Q). */
int mf4d_set_queries(mf4d_ctx *ctx, int Q, const float *crit, const int32_t *qxyzt, int64_t S,
                     int where);

/* Tile of the batched grower: bx * by * bz * bt = 512 voxel-steps, each a
 * power of two (default 8 x 4 x 4 x 4); one thread per voxel-step of a tile.
 * Errors: MF4D_ERR_ARG. */
int mf4d_set_batched_tile(mf4d_ctx *ctx, int bx, int by, int bz, int bt);

/* Grow every query (as mf4d_grow grows one, Section 1's output for each)
 * and write the results: fplanes uint32 [X*Y*Z*T][8] in
 * canonical voxel order, query q in bit (q & 31) of word (q >> 5); pplanes
 * uint32 [T][P][8] likewise (NULL allowed when no particles are loaded).
 * Planes q >= Q are zero.  Device outputs are grown in place.
 * Errors: MF4D_ERR_STATE (no field or no queries), MF4D_ERR_ARG (buffers
 * too small), MF4D_ERR_OOM, MF4D_ERR_HIP. */
int mf4d_grow_batched(mf4d_ctx *ctx, uint32_t *fplanes, size_t fwords, uint32_t *pplanes,
                      size_t pwords, int where, mf4d_stats *out);

/* The planes of the last mf4d_grow_batched call that was given no output
 * buffers (fplanes and pplanes NULL, fwords and pwords 0): such a call grows
 * into planes the context owns (allocated on first use: 32 bytes per
 * voxel-step and per particle-step), and this call copies them out in the
 * layouts of mf4d_grow_batched.  pdst may be NULL (then pwords is ignored).
 * Waits for the copies.
 * Errors: MF4D_ERR_STATE (no batched grow into context planes since the
 * last load or query change), MF4D_ERR_ARG (a buffer too small). */
int mf4d_read_batched(mf4d_ctx *ctx, uint32_t *fdst, size_t fwords, uint32_t *pdst, size_t pwords,
                      int where);

/* ---- brick-activity predictor --------------------------------------------
 * A 3-layer 3D convolutional network (8 -> 16 -> 16 -> 1 channels, 3x3x3,
 * zero "same" padding, ReLU, logits) over the grid of bricks of 8^3 voxels of
 * each timestep.  Inputs are per brick-step (field min, max, mean minus the
 * field lower bound; log1p(particle-steps) / 4) at t and at t-1, in bf16
 * channels-last [T][Db][Hb][Wb][16] (channels 8..15 zero).  It predicts
 * whether a brick-step will hold a member of the grown feature; the grower
 * uses it only to choose which candidate tiles to test before the rounds (the
 * rest are tested by the first sweep that reaches them), so the result never
 * depends on it.  Weights bf16 on the matrix cores with fp32 accumulation
 * (bf16 hidden activations for inference, fp32 ones for training); fp32
 * master parameters, Adam.  Parameter layout (fp32, 10833 values): per
 * layer W [cout][cin][3][3][3] then b [cout]. */

/* The network has no counterpart in the paper; its inputs summarise the
 * field and point samples of Section 3.1 per brick-step.
 * Number of parameters (10833). */
int mf4d_net_num_params(void);

/* Create a network with zero parameters on `device`, ordering its work on
 * `hip_stream`.  Errors: MF4D_ERR_ARG, MF4D_ERR_OOM, MF4D_ERR_HIP. */
int mf4d_net_create(mf4d_net **out, int device, void *hip_stream);
void mf4d_net_destroy(mf4d_net *net);
const char *mf4d_net_last_error(void);

/* Copy parameters in (resets the Adam state) or out.  where: MF4D_HOST or
 * MF4D_DEVICE. */
int mf4d_net_set_params(mf4d_net *net, const float *params, int where);
int mf4d_net_get_params(mf4d_net *net, float *params, int where);

/* Logits fp32 [N][D][H][W] of inputs x bf16 [N][D][H][W][16] (channels 0..7
 * are the network's inputs, 8..15 are ignored) at inference precision: bf16
 * hidden activations; device pointers only.  Errors: MF4D_ERR_ARG,
 * MF4D_ERR_UNSUPPORTED (>= 2^31 positions). */
int mf4d_net_forward(mf4d_net *net, const uint16_t *x, int N, int D, int H, int W, float *logits,
                     int where);

/* Gradients (fp32, parameter layout, device) of the mean binary cross entropy
 * with positive weight `pos_weight` against labels y uint8 [N][D][H][W];
 * *loss receives the loss.  Training precision: fp32 hidden activations and
 * layer gradients (operands split into bf16 pieces on the matrix cores).
 * Device pointers only. */
int mf4d_net_grad(mf4d_net *net, const uint16_t *x, const uint8_t *y, int N, int D, int H, int W,
                  float pos_weight, float *grads, float *loss, int where);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on that loss; device pointers;
 * *loss (nullable) receives the loss before the step. */
int mf4d_net_train_step(mf4d_net *net, const uint16_t *x, const uint8_t *y, int N, int D, int H,
                        int W, float pos_weight, float lr, float *loss);

/* The network's three kernels as separate calls, for a trainer that drives
 * them itself.  mf4d_nn_forward is mf4d_net_forward.  mf4d_nn_backward is
 * mf4d_net_grad that also writes, when dx is not NULL, the gradient of the
 * loss with respect to the inputs x as fp32 [N][D][H][W][16] (channels 8..15
 * are unused inputs and read 0).  mf4d_nn_adam_step applies one Adam step
 * (beta 0.9 / 0.999, eps 1e-8, learning rate lr) with the gradients `grads`
 * (fp32, parameter layout, device; NULL: those of the last mf4d_nn_backward
 * or mf4d_net_grad call).  Device pointers only (where = MF4D_DEVICE).
 * Errors: MF4D_ERR_ARG, MF4D_ERR_UNSUPPORTED, MF4D_ERR_OOM, MF4D_ERR_HIP. */
int mf4d_nn_forward(mf4d_net *net, const uint16_t *x, int N, int D, int H, int W, float *logits,
                    int where);
int mf4d_nn_backward(mf4d_net *net, const uint16_t *x, const uint8_t *y, int N, int D, int H, int W,
                     float pos_weight, float *grads, float *dx, float *loss, int where);
int mf4d_nn_adam_step(mf4d_net *net, const float *grads, float lr, int where);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * logits as mf4d_nn_forward, from the same kernels, with the two hidden
 * activations in a static per-GPU scratch array of 16 MiB instead of buffers
 * the network allocates, so the call allocates and frees nothing.  At most
 * 2^18 positions (N*D*H*W <= 262144).  Stream-ordered on the network's
 * stream; returns without waiting.  Every call on one GPU shares that GPU's
 * scratch, so calls that overlap on one GPU (another stream, another thread,
 * another network on the same device) race and must be serialised by the
 * caller.  Device pointers only.
 * Errors: MF4D_ERR_ARG, MF4D_ERR_RANGE (more positions than the scratch
 * holds), MF4D_ERR_UNSUPPORTED, MF4D_ERR_STATE, MF4D_ERR_HIP. */
int mf4d_nn_forward_noalloc(mf4d_net *net, const uint16_t *x, int N, int D, int H, int W, float *logits,
                            int where);

/* Brick grid of the loaded field: dims4 = (T, Db, Hb, Wb). */
int mf4d_brick_dims(mf4d_ctx *ctx, int *dims4);

/* Network inputs for the loaded data under the current criteria (layout
 * above), n >= T*Db*Hb*Wb*16 elements. */
int mf4d_features(mf4d_ctx *ctx, uint16_t *dst, size_t n, int where);

/* Labels of the last grow: uint8 [T][Db][Hb][Wb], 1 = the brick-step holds a
 * member voxel-step. */
int mf4d_brick_labels(mf4d_ctx *ctx, uint8_t *dst, size_t n, int where);

/* Use `net` (NULL: none) to choose the tiles tested before the rounds: a
 * candidate tile is tested up front when one of its brick-steps has a logit
 * >= logit_threshold.  The context keeps the pointer; the net must outlive
 * its use.  Errors: MF4D_ERR_ARG (NaN threshold). */
int mf4d_set_predictor(mf4d_ctx *ctx, mf4d_net *net, float logit_threshold);

/* Choose the scheduler of the context's grows.  MF4D_SCHEDULER_PLAIN (the
 * default): params must be NULL and nbytes 0.  MF4D_SCHEDULER_LEARNED: params
 * holds, on the host, the network's fp32 parameters (mf4d_net_num_params()
 * values, layout above) followed by one fp32 logit threshold, nbytes = 4 *
 * (mf4d_net_num_params() + 1); the context keeps its own copy of the network
 * (on its device and stream) and uses it as mf4d_set_predictor does.  No
 * scheduler changes the grown set (the least fixed point of the coupled
 * graph is unique; a verification round and the plain rounds judge it).
 * Errors: MF4D_ERR_ARG (unknown kind, bad size, NaN threshold),
 * MF4D_ERR_OOM, MF4D_ERR_HIP. */
int mf4d_set_scheduler(mf4d_ctx *ctx, int kind, const void *params, size_t nbytes);

/* Statistics of the last grow, including member counts of the last reads. */
int mf4d_last_stats(mf4d_ctx *ctx, mf4d_stats *out);

/* ---- 4D SLIC clustering of the loaded point and field samples (Section 3.2) ----
 *
 * Samples: one per voxel-step, at the voxel centre (x+0.5, y+0.5, z+0.5), time
 * t, value f; one per loaded particle-step, at its position, time t, value a.
 * A sample with a non-finite position or value is not clustered (label -1).
 * Centres start on a kx x ky x kz x kt grid of intervals C_d = E_d / k_d with
 * E = (X, Y, Z, T) (Section 3.2.1); every sample first joins its grid cell's
 * centre (the nearest).  An iteration recomputes each centre as the mean
 * location of its samples, the mean point value and the mean field value
 * (Section 3.2.2), then assigns each sample to the centre with the smallest
 * D_f = w_f |f - f_c| + w_d S_st or D_p = w_p |a - p_c| + w_d S_st (Section
 * 3.2.3), S_st being the 4D distance with time scaled by c_f (Section 3.2.1),
 * among the centres whose 2C_1 x 2C_2 x 2C_3 x 2C_4 window (Section 3.2.2)
 * holds the sample -- searched among the centres seeded in the 3^4 grid cells
 * around the sample's own; ties go to the lowest centre id, and a sample with
 * no candidate keeps its centre.  Centre id = ((ct*kz + cz)*ky + cy)*kx + cx.
 * Means come from exact integer sums of coordinates and values quantised to
 * 2^-20 (so they do not depend on the order of additions); distances are IEEE
 * fp32 operations in a fixed order.  The loop stops when no centre value
 * changed by more than eps times its previous magnitude (the relative-change
 * test of Section 3.2.2), or after max_iter assignment passes. */

/* k4 = (kx, ky, kz, kt), each in [1, 4096], at most 2^24 centres; weights and
 * c_f finite and >= 0; eps >= 0; max_iter in [0, 100000].
 * Errors: MF4D_ERR_ARG, MF4D_ERR_OOM. */
int mf4d_slic_set_params(mf4d_ctx *ctx, const int *k4, float w_d, float w_f, float w_p, float c_f,
                         double eps, int max_iter);

/* Cluster the loaded field (and particles, if loaded).  *iterations (nullable)
 * receives the number of assignment passes.  Waits for the device.
 * Errors: MF4D_ERR_STATE (no field or no parameters), MF4D_ERR_UNSUPPORTED (a
 * dimension >= 2048, or 2^31 samples or more), MF4D_ERR_RANGE (a coordinate
 * or value with magnitude >= 2048: the exact sums could overflow; the labels
 * are then not defined), MF4D_ERR_OOM, MF4D_ERR_HIP. */
int mf4d_slic_run(mf4d_ctx *ctx, int *iterations);

/* Labels of the last run: field int32 [T][Z][Y][X] (nf >= X*Y*Z*T) and point
 * int32 [T][P] (np >= T*P); either pointer may be NULL.  With MF4D_DEVICE the
 * copies are ordered on the context's stream and the call returns at once.
 * Errors: MF4D_ERR_STATE (no run), MF4D_ERR_ARG (too small). */
int mf4d_slic_read_labels(mf4d_ctx *ctx, int32_t *field_labels, size_t nf, int32_t *point_labels,
                          size_t np, int where);

/* Centres of the last run: fp64 [K][6] as (x, y, z, t, p_c, f_c) and int64
 * [K][2] sample counts (field, point); either pointer may be NULL; K >=
 * kx*ky*kz*kt.  A centre that never had samples of a type keeps 0 for that
 * type's value; one without samples keeps its seed location.
 * Errors: MF4D_ERR_STATE (no run), MF4D_ERR_ARG. */
int mf4d_slic_read_centres(mf4d_ctx *ctx, double *centres, int64_t *counts, size_t K, int where);

/* Merge the centres of the last run into features (Section 3.3): two centres
 * match when, for each sample type, neither has samples of it or both do and
 * their means differ by at most eps_m times the larger magnitude (location is
 * ignored); a centre without samples matches nothing.  Features are the
 * transitive groups of matching centres, each named by its lowest centre id
 * (a background "supercluster" is simply the group its centres form).
 * *n_features (nullable) receives their number.  Waits for the device.
 * Errors: MF4D_ERR_STATE (no run), MF4D_ERR_ARG (eps_m not finite or < 0). */
int mf4d_slic_merge(mf4d_ctx *ctx, double eps_m, int *n_features);

/* Result of the last merge: the feature of each centre, int32 [K] (-1: a
 * centre without samples), and per feature id fp64 [K][14]: field and point
 * sample counts, mean field and point values (from the exact sums of the
 * clustering), population standard deviations of the field and point values,
 * then the least and greatest x, y, z and t of its samples (the extent of
 * Section 3.3's feature list); rows of ids that name no feature hold zeros.
 * Either pointer may be NULL.  Errors: MF4D_ERR_STATE (no merge since the
 * last run), MF4D_ERR_ARG (K too small). */
int mf4d_slic_read_features(mf4d_ctx *ctx, int32_t *feature_of_centre, double *stats, size_t K,
                            int where);

/* Trajectory segments of the merged features (Section 3.4): the feature id
 * of point sample (t, p) where the same particle has that feature at t - 1
 * or t + 1, else -1, as int32 [T][P] in dst (n >= T*P).  A trajectory that
 * passes through several features is thereby split into pieces of two or
 * more consecutive steps each.  Uses the labels of the last run and the
 * features of the last merge.  Stream ordering as mf4d_slic_read_labels.
 * Errors: MF4D_ERR_STATE (no merge since the last run, or a run without
 * point samples), MF4D_ERR_ARG (dst NULL or too small). */
int mf4d_slic_read_segments(mf4d_ctx *ctx, int32_t *dst, size_t n, int where);

#ifdef __cplusplus
}
#endif

#endif /* MF4D_H */
