/*
 * Reference breadth-first grower for the coupled point + field graph.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the CPU oracle that the GPU
 * library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header or table with the GPU library.
 *
 * What it computes (the plain definition, written out):
 *   Nodes are voxel-steps v = (x, y, z, t) of the field grid (Section 3.1,
 *   F(t) = {x_f, y_f, z_f, v_f(t)}) and particle-steps q = (i, t) of the
 *   point data (Section 3.1, P(t) = {x_p(t), y_p(t), z_p(t), v_p(t)}).
 *   Membership criterion per sample type (the per-type value terms of the
 *   distance metrics D_f and D_p, Section 3.2.3, read as inclusive bands):
 *       A_f(v) <=> f_lo <= f(v) <= f_hi,   A_p(q) <=> a_lo <= a(q) <= a_hi
 *   compared in fp32 on the stored values (NaN is never admissible).
 *   Undirected edges:
 *     - the six spatial grid neighbours of a voxel (each grid location has a
 *       distinct set of neighbours, Section 3.1), no wrap-around;
 *     - the same voxel at t-1 and t+1;
 *     - a particle-step and the voxel whose volume holds it (the field-to-
 *       point index of Section 3.1): voxel i covers [i, i+1) per axis in
 *       voxel units; a step with any coordinate outside [0, dim) or NaN lies
 *       in no voxel;
 *     - a particle-step and the same particle at t-1 and t+1 (trajectories
 *       connect points between timesteps, Section 1).
 *   Result M = the nodes reachable from the admissible seeds inside the
 *   subgraph induced on admissible nodes.  Seeds that are not admissible are
 *   dropped and counted.
 *   Particles at their own temporal rate (oracle_grow_rate): the particles
 *   hold Tp steps, r per field step; particle step tau lies at time tau / r
 *   in field steps and couples with a voxel of field step floor(tau / r),
 *   the step whose interval [t, t+1) holds that time.  Trajectory edges join
 *   consecutive particle steps.  r = 1 and Tp = T is the plain case.
 *   Forward-only (causal) coupling, forward_only = 1:
 *   the trajectory edge leads only from (i, t) to (i, t+1), so membership
 *   travels along a trajectory forward in time; every other edge stays
 *   undirected, and M is the set reachable along the directed edges.
 *
 * Algorithm: textbook FIFO breadth-first search.  The voxel -> particle-step
 * index is a counting sort of particle-steps by voxel id (CSR).
 *
 * Output layouts: field mask bit ((t*Z + z)*Y + y)*X + x, word = bit >> 5,
 * LSB first; particle mask uint8 [Tp][P].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_RANGE (-2)
#define OR_ERR_OOM (-3)

#define NO_VOXEL UINT32_MAX

static int in_band(float v, float lo, float hi) { return lo <= v && v <= hi; }

/* Voxel (spatial part) holding a stored fp32 position, or -1. */
static int64_t voxel_of(const float *p, int64_t X, int64_t Y, int64_t Z)
{
    float cx = floorf(p[0]), cy = floorf(p[1]), cz = floorf(p[2]);
    if (!(cx >= 0.0f && cx < (float)X)) return -1;
    if (!(cy >= 0.0f && cy < (float)Y)) return -1;
    if (!(cz >= 0.0f && cz < (float)Z)) return -1;
    return ((int64_t)cz * Y + (int64_t)cy) * X + (int64_t)cx;
}

typedef struct {
    uint64_t *v;
    size_t head, tail, cap;
} fifo_t;

static int fifo_push(fifo_t *q, uint64_t n)
{
    if (q->tail == q->cap) {
        size_t nc = q->cap ? q->cap * 2 : 1024;
        uint64_t *nv = (uint64_t *)realloc(q->v, nc * sizeof(uint64_t));
        if (!nv) return OR_ERR_OOM;
        q->v = nv;
        q->cap = nc;
    }
    q->v[q->tail++] = n;
    return OR_OK;
}

static int test_and_set(uint64_t *bits, uint64_t i)
{
    uint64_t m = (uint64_t)1 << (i & 63);
    if (bits[i >> 6] & m) return 0;
    bits[i >> 6] |= m;
    return 1;
}

/*
 * stats[0] = |M ∩ voxels|, stats[1] = |M ∩ particle-steps|,
 * stats[2] = dropped (inadmissible) seed entries,
 * stats[3] = D, the largest BFS level (0 when M is empty),
 * stats[4] = number of admissible seed entries.
 * Returns 0, OR_ERR_ARG, OR_ERR_RANGE (a seed outside the grid) or OR_ERR_OOM.
 */
int oracle_grow_rate(const float *field, int64_t X, int64_t Y, int64_t Z, int64_t T,
                     const float *xyz, const float *attr, int64_t P, int64_t Tp, int64_t r,
                     float f_lo, float f_hi, float a_lo, float a_hi,
                     const int32_t *seeds, int64_t S, int forward_only,
                     uint32_t *fmask, uint8_t *pmask, int64_t *stats)
{
    if (X <= 0 || Y <= 0 || Z <= 0 || T <= 0 || P < 0 || S < 0) return OR_ERR_ARG;
    if (r < 1 || Tp < 1 || Tp > r * T) return OR_ERR_ARG;
    if (!field || !fmask || !stats || (S > 0 && !seeds)) return OR_ERR_ARG;
    if (P > 0 && (!xyz || !attr || !pmask)) return OR_ERR_ARG;
    const uint64_t XY = (uint64_t)X * Y, XYZ = XY * Z, V = XYZ * T;
    const uint64_t Q = (uint64_t)P * Tp;
    if (V >= (uint64_t)UINT32_MAX || Q >= (uint64_t)UINT32_MAX) return OR_ERR_ARG;
    for (int64_t s = 0; s < S; ++s) {
        const int32_t *sd = seeds + 4 * s;
        if (sd[0] < 0 || sd[0] >= X || sd[1] < 0 || sd[1] >= Y || sd[2] < 0 ||
            sd[2] >= Z || sd[3] < 0 || sd[3] >= T)
            return OR_ERR_RANGE;
    }

    int rc = OR_ERR_OOM;
    uint32_t *bin = NULL, *start = NULL, *order = NULL;
    uint64_t *visF = NULL, *visP = NULL;
    fifo_t fifo = {0};

    visF = (uint64_t *)calloc(V / 64 + 1, sizeof(uint64_t));
    visP = (uint64_t *)calloc(Q / 64 + 1, sizeof(uint64_t));
    if (!visF || !visP) goto done;

    if (Q > 0) {
        /* Voxel-step of every particle-step. */
        bin = (uint32_t *)malloc(Q * sizeof(uint32_t));
        start = (uint32_t *)calloc(V + 1, sizeof(uint32_t));
        order = (uint32_t *)malloc(Q * sizeof(uint32_t));
        if (!bin || !start || !order) goto done;
        for (uint64_t t = 0; t < (uint64_t)Tp; ++t)
            for (uint64_t i = 0; i < (uint64_t)P; ++i) {
                uint64_t q = t * P + i;
                int64_t s = voxel_of(xyz + 3 * q, X, Y, Z);
                uint64_t tf = t / (uint64_t)r; /* the field step holding time t / r */
                bin[q] = s < 0 ? NO_VOXEL : (uint32_t)(tf * XYZ + (uint64_t)s);
            }
        /* Counting sort of particle-steps by voxel: start[v]..start[v+1]. */
        for (uint64_t q = 0; q < Q; ++q)
            if (bin[q] != NO_VOXEL) start[bin[q] + 1]++;
        for (uint64_t v = 0; v < V; ++v) start[v + 1] += start[v];
        uint32_t *fill = (uint32_t *)malloc(V * sizeof(uint32_t));
        if (!fill) goto done;
        memcpy(fill, start, V * sizeof(uint32_t));
        for (uint64_t q = 0; q < Q; ++q)
            if (bin[q] != NO_VOXEL) order[fill[bin[q]]++] = (uint32_t)q;
        free(fill);
    }

    int64_t dropped = 0, kept = 0;
    for (int64_t s = 0; s < S; ++s) {
        const int32_t *sd = seeds + 4 * s;
        uint64_t v = (uint64_t)sd[3] * XYZ + (uint64_t)sd[2] * XY + (uint64_t)sd[1] * X + sd[0];
        if (!in_band(field[v], f_lo, f_hi)) { dropped++; continue; }
        kept++;
        if (test_and_set(visF, v) && fifo_push(&fifo, v)) goto done;
    }

    /* Node id: voxel-step v < V, particle-step q as V + q. */
    int64_t depth = 0;
    while (fifo.head < fifo.tail) {
        size_t layer_end = fifo.tail;
        while (fifo.head < layer_end) {
            uint64_t n = fifo.v[fifo.head++];
            if (n < V) {
                uint64_t v = n;
                uint64_t x = v % X, y = (v / X) % Y, z = (v / XY) % Z, t = v / XYZ;
                uint64_t nb[8];
                int k = 0;
                if (x > 0) nb[k++] = v - 1;
                if (x + 1 < (uint64_t)X) nb[k++] = v + 1;
                if (y > 0) nb[k++] = v - X;
                if (y + 1 < (uint64_t)Y) nb[k++] = v + X;
                if (z > 0) nb[k++] = v - XY;
                if (z + 1 < (uint64_t)Z) nb[k++] = v + XY;
                if (t > 0) nb[k++] = v - XYZ;
                if (t + 1 < (uint64_t)T) nb[k++] = v + XYZ;
                for (int j = 0; j < k; ++j)
                    if (in_band(field[nb[j]], f_lo, f_hi) && test_and_set(visF, nb[j]))
                        if (fifo_push(&fifo, nb[j])) goto done;
                if (Q > 0)
                    for (uint32_t e = start[v]; e < start[v + 1]; ++e) {
                        uint64_t q = order[e];
                        if (in_band(attr[q], a_lo, a_hi) && test_and_set(visP, q))
                            if (fifo_push(&fifo, V + q)) goto done;
                    }
            } else {
                uint64_t q = n - V;
                uint64_t t = q / P;
                if (bin[q] != NO_VOXEL && in_band(field[bin[q]], f_lo, f_hi) &&
                    test_and_set(visF, bin[q]))
                    if (fifo_push(&fifo, bin[q])) goto done;
                if (!forward_only && t > 0 && in_band(attr[q - P], a_lo, a_hi) &&
                    test_and_set(visP, q - P))
                    if (fifo_push(&fifo, V + q - P)) goto done;
                if (t + 1 < (uint64_t)Tp && in_band(attr[q + P], a_lo, a_hi) &&
                    test_and_set(visP, q + P))
                    if (fifo_push(&fifo, V + q + P)) goto done;
            }
        }
        if (fifo.tail > layer_end) depth++;
    }

    int64_t mf = 0, mp = 0;
    memset(fmask, 0, ((V + 31) / 32) * sizeof(uint32_t));
    for (uint64_t v = 0; v < V; ++v)
        if (visF[v >> 6] >> (v & 63) & 1) {
            fmask[v >> 5] |= (uint32_t)1 << (v & 31);
            mf++;
        }
    for (uint64_t q = 0; q < Q; ++q) {
        pmask[q] = (uint8_t)(visP[q >> 6] >> (q & 63) & 1);
        mp += pmask[q];
    }
    stats[0] = mf;
    stats[1] = mp;
    stats[2] = dropped;
    stats[3] = depth;
    stats[4] = kept;
    rc = OR_OK;
done:
    free(fifo.v);
    free(bin);
    free(start);
    free(order);
    free(visF);
    free(visP);
    return rc;
}

/* Particles at the field's rate (Tp = T, r = 1). */
int oracle_grow_dir(const float *field, int64_t X, int64_t Y, int64_t Z, int64_t T,
                    const float *xyz, const float *attr, int64_t P,
                    float f_lo, float f_hi, float a_lo, float a_hi,
                    const int32_t *seeds, int64_t S, int forward_only,
                    uint32_t *fmask, uint8_t *pmask, int64_t *stats)
{
    return oracle_grow_rate(field, X, Y, Z, T, xyz, attr, P, T, 1, f_lo, f_hi, a_lo, a_hi, seeds, S,
                            forward_only, fmask, pmask, stats);
}

/* Both trajectory directions (undirected coupling). */
int oracle_grow(const float *field, int64_t X, int64_t Y, int64_t Z, int64_t T,
                const float *xyz, const float *attr, int64_t P,
                float f_lo, float f_hi, float a_lo, float a_hi,
                const int32_t *seeds, int64_t S,
                uint32_t *fmask, uint8_t *pmask, int64_t *stats)
{
    return oracle_grow_dir(field, X, Y, Z, T, xyz, attr, P, f_lo, f_hi, a_lo, a_hi, seeds, S, 0,
                           fmask, pmask, stats);
}
