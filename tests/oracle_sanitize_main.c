/* Drives the C breadth-first oracle (oracle/grow_bfs.c) over many small
 * seeded instances so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer can catch out-of-bounds accesses, leaks and
 * undefined behaviour.  Instances mix the edge cases the oracle handles:
 * NaN and infinite values, particle positions outside the grid or NaN, no
 * particles, unit dimensions, several particle steps per field step,
 * forward-only coupling, duplicate seeds, inadmissible seeds, a seed outside
 * the grid (an error return).  Exits 0 when every call returned what it
 * should. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_grow_rate(const float *field, int64_t X, int64_t Y, int64_t Z, int64_t T, const float *xyz,
                     const float *attr, int64_t P, int64_t Tp, int64_t r, float f_lo, float f_hi, float a_lo,
                     float a_hi, const int32_t *seeds, int64_t S, int forward_only, uint32_t *fmask,
                     uint8_t *pmask, int64_t *stats);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint32_t next(void) {
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(state >> 33);
}
static float unit(void) { return (float)(next() & 0xFFFFFF) / 16777216.0f; }

int main(void) {
    int failures = 0;
    for (int it = 0; it < 400; ++it) {
        const int64_t X = 1 + next() % 7, Y = 1 + next() % 6, Z = 1 + next() % 5, T = 1 + next() % 4;
        const int64_t P = (it % 5 == 0) ? 0 : next() % 40;
        const int64_t r = 1 + next() % 3;
        const int64_t Tp = r * T - (int64_t)(next() % r);
        const int64_t V = X * Y * Z * T, Q = P * Tp;
        float *field = malloc((size_t)V * sizeof(float));
        float *xyz = malloc((size_t)(Q ? Q : 1) * 3 * sizeof(float));
        float *attr = malloc((size_t)(Q ? Q : 1) * sizeof(float));
        for (int64_t i = 0; i < V; ++i) {
            const uint32_t k = next() % 50;
            field[i] = k == 0 ? NAN : (k == 1 ? INFINITY : (k == 2 ? -INFINITY : unit()));
        }
        for (int64_t i = 0; i < Q; ++i) {
            const float dims[3] = {(float)X, (float)Y, (float)Z};
            for (int a = 0; a < 3; ++a) {
                const uint32_t k = next() % 30;
                xyz[3 * i + a] = k == 0 ? NAN : (k == 1 ? -0.5f : (k == 2 ? dims[a] : unit() * dims[a]));
            }
            attr[i] = (next() % 40 == 0) ? NAN : unit();
        }
        const int64_t S = next() % 6;
        int32_t *seeds = malloc((size_t)(S ? S : 1) * 4 * sizeof(int32_t));
        for (int64_t s = 0; s < S; ++s) {
            seeds[4 * s] = next() % X;
            seeds[4 * s + 1] = next() % Y;
            seeds[4 * s + 2] = next() % Z;
            seeds[4 * s + 3] = next() % T;
        }
        if (S > 1) for (int a = 0; a < 4; ++a) seeds[4 + a] = seeds[a];  /* a duplicate */
        const int bad = S > 0 && it % 7 == 3;
        if (bad) seeds[0] = (int32_t)X;  /* outside the grid */
        uint32_t *fmask = calloc((size_t)(V + 31) / 32 + 1, sizeof(uint32_t));
        uint8_t *pmask = calloc((size_t)(Q ? Q : 1), 1);
        int64_t stats[5] = {0, 0, 0, 0, 0};
        const float lo = it % 3 == 0 ? -INFINITY : unit() * 0.8f;
        const int rc = oracle_grow_rate(field, X, Y, Z, T, P ? xyz : NULL, P ? attr : NULL, P, Tp, r, lo,
                                        INFINITY, lo * 0.9f, INFINITY, seeds, S, it & 1, fmask,
                                        P ? pmask : NULL, stats);
        if (bad ? rc != -2 : rc != 0) {
            fprintf(stderr, "instance %d: return %d\n", it, rc);
            ++failures;
        }
        if (!bad && (stats[0] > V || stats[1] > Q || stats[2] > S)) {
            fprintf(stderr, "instance %d: statistics out of range\n", it);
            ++failures;
        }
        free(field);
        free(xyz);
        free(attr);
        free(seeds);
        free(fmask);
        free(pmask);
    }
    printf("%d failures\n", failures);
    return failures ? 1 : 0;
}
