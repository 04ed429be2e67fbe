/*
 * Seeded synthetic inputs for the GP-tree evaluation path.
 *
 * This module only produces input data: the fitness-case table and
 * populations of prefix-linear trees (one byte per node, root first).
 * It holds none of the evaluation, fitness, crossover or selection
 * arithmetic; the oracle and the HIP library each implement those on
 * their own and both consume what this file writes.
 *
 * Token values (the paper only says "8 bit opcode", Sec. 2.1/2.2):
 *   0 ADD, 1 SUB, 2 MUL, 3 DIV, 4 X.
 *
 * Generators:
 *   wl_cases       evenly spaced x in [-1,1] and the Sextic target
 *                  x^6 - 2x^4 + x^2 (Sec. 3, Table 1), computed in
 *                  binary64 at the binary32 x and rounded once.
 *   wl_rhh         Koza ramped half-and-half, depths dmin..dmax
 *                  (Table 1: initial population, depth 2 to 6).
 *   wl_random_tree a uniformly random binary tree with a given odd
 *                  number of nodes (Lukasiewicz word + cycle lemma),
 *                  ops drawn uniformly; the paper notes evolved trees
 *                  are shaped roughly like random trees (Sec. 2.2).
 *   wl_random_pop  many such trees, in parallel (pthreads), written
 *                  straight into a caller buffer.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

#define WL_ADD 0
#define WL_SUB 1
#define WL_MUL 2
#define WL_DIV 3
#define WL_X 4

/* splitmix64 (Steele, Lea, Flood 2014) - generator-side randomness only */
static inline uint64_t sm64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* xoshiro256** (Blackman, Vigna 2018) seeded from splitmix64 */
typedef struct { uint64_t s[4]; } wl_rng;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void rng_seed(wl_rng *r, uint64_t seed, uint64_t stream)
{
    uint64_t s = seed ^ (stream * 0xD1B54A32D192ED03ull + 0x2545F4914F6CDD1Dull);
    for (int i = 0; i < 4; i++) r->s[i] = sm64(&s);
}

static inline uint64_t rng_next(wl_rng *r)
{
    uint64_t *s = r->s;
    uint64_t res = rotl64(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl64(s[3], 45);
    return res;
}

/* uniform integer in [0, n) for n < 2^32 (multiply-shift, bias < n/2^32) */
static inline uint32_t rng_below32(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * n) >> 32);
}

static inline double rng_unit(wl_rng *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* ---------------------------------------------------------------- cases */

void wl_cases(int32_t n, float *x, float *y)
{
    for (int32_t i = 0; i < n; i++) {
        double xd = (n == 1) ? 0.0 : -1.0 + 2.0 * (double)i / (double)(n - 1);
        float xf = (float)xd;
        double v = (double)xf;
        double v2 = v * v, v4 = v2 * v2, v6 = v4 * v2;
        x[i] = xf;
        y[i] = (float)(v6 - 2.0 * v4 + v2);
    }
}

/* ------------------------------------------------- ramped half-and-half */

typedef struct { uint8_t *buf; uint64_t len, cap; } wl_out;

static int out_put(wl_out *o, uint8_t t)
{
    if (o->len >= o->cap) return -1;
    o->buf[o->len++] = t;
    return 0;
}

static int rhh_node(wl_out *o, wl_rng *r, int depth, int dmax, int full)
{
    int term;
    if (depth >= dmax) term = 1;
    else if (depth == 0) term = 0;
    else if (full) term = 0;
    else term = (rng_next(r) % 5u) == 0; /* grow: terminal w.p. 1/5 */
    if (term) return out_put(o, WL_X);
    if (out_put(o, (uint8_t)(rng_next(r) & 3u))) return -1;
    if (rhh_node(o, r, depth + 1, dmax, full)) return -1;
    return rhh_node(o, r, depth + 1, dmax, full);
}

/* M trees; tree i has max depth dmin + i % (dmax-dmin+1), full when
 * (i / (dmax-dmin+1)) is even, grow otherwise.  off has M+1 entries.
 * Returns total bytes, or -1 when cap is too small. */
int64_t wl_rhh(uint64_t seed, int32_t M, int32_t dmin, int32_t dmax,
               uint8_t *buf, uint64_t cap, uint64_t *off)
{
    wl_out o = {buf, 0, cap};
    int span = dmax - dmin + 1;
    off[0] = 0;
    for (int32_t i = 0; i < M; i++) {
        wl_rng r;
        rng_seed(&r, seed, (uint64_t)i);
        int d = dmin + i % span;
        int full = ((i / span) % 2) == 0;
        if (rhh_node(&o, &r, 0, d, full)) return -1;
        off[i + 1] = o.len;
    }
    return (int64_t)o.len;
}

/* ------------------------------------------------ uniform random trees */

/* One uniformly random binary tree with n (odd) nodes into dst.
 * A uniformly random arrangement of k=(n-1)/2 ops and k+1 leaves is drawn
 * sequentially; the cycle lemma (Dvoretzky-Motzkin) says exactly one
 * rotation of it is a valid prefix word: the one starting at the first
 * position where the running sum (op +1, leaf -1) is minimal. */
void wl_random_tree(uint64_t seed, uint64_t stream, uint64_t n, uint8_t *dst)
{
    wl_rng r;
    rng_seed(&r, seed, stream);
    if (n <= 1) { if (n == 1) dst[0] = WL_X; return; }
    uint64_t k = (n - 1) / 2;
    uint64_t ops_left = k, left = n;
    int64_t run = 0, best = 0;
    uint64_t best_at = 0;
    uint64_t w = 0;
    int wbits = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t u;
        if (wbits == 0) { w = rng_next(&r); wbits = 2; }
        u = (uint32_t)(w >> 32); w <<= 32; wbits--;
        int is_op;
        if (left > 0xFFFFFFFFull) {
            is_op = (double)u * (double)left < (double)ops_left * 4294967296.0;
        } else {
            is_op = rng_below32(u, (uint32_t)left) < ops_left;
        }
        left--;
        if (is_op) { ops_left--; dst[i] = 0; run++; }
        else { dst[i] = WL_X; run--; }
        /* running sum after position i is the prefix before position i+1 */
        if (i + 1 < n && run < best) { best = run; best_at = i + 1; }
    }
    /* rotate left by best_at */
    if (best_at) {
        uint64_t a = best_at;
        /* three reversals */
        for (uint64_t i = 0, j = a - 1; i < j; i++, j--) { uint8_t t = dst[i]; dst[i] = dst[j]; dst[j] = t; }
        for (uint64_t i = a, j = n - 1; i < j; i++, j--) { uint8_t t = dst[i]; dst[i] = dst[j]; dst[j] = t; }
        for (uint64_t i = 0, j = n - 1; i < j; i++, j--) { uint8_t t = dst[i]; dst[i] = dst[j]; dst[j] = t; }
    }
    /* label ops uniformly */
    uint64_t bits = 0;
    int nb = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (dst[i] == WL_X) continue;
        if (nb == 0) { bits = rng_next(&r); nb = 32; }
        dst[i] = (uint8_t)(bits & 3u);
        bits >>= 2; nb--;
    }
}

/* sizes: odd node counts, log-uniform in [lo, hi] */
void wl_loguniform_sizes(uint64_t seed, int32_t M, double lo, double hi, uint64_t *sizes)
{
    wl_rng r;
    rng_seed(&r, seed, 0xABCDEFull);
    double a = log(lo), b = log(hi);
    for (int32_t i = 0; i < M; i++) {
        double s = exp(a + (b - a) * rng_unit(&r));
        uint64_t n = (uint64_t)llround(s);
        if (n < 1) n = 1;
        if ((n & 1) == 0) n = (n + 1 <= (uint64_t)hi) ? n + 1 : n - 1;
        sizes[i] = n;
    }
}

typedef struct {
    uint64_t seed;
    const uint64_t *off;
    int32_t M;
    uint8_t *buf;
    int32_t next;
    pthread_mutex_t mu;
} pop_job;

static void *pop_worker(void *arg)
{
    pop_job *j = (pop_job *)arg;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        int32_t t = j->next++;
        pthread_mutex_unlock(&j->mu);
        if (t >= j->M) break;
        wl_random_tree(j->seed, 0x100000000ull + (uint64_t)t, j->off[t + 1] - j->off[t], j->buf + j->off[t]);
    }
    return NULL;
}

/* Fill buf (sized off[M]) with M random trees, tree t occupying
 * [off[t], off[t+1]).  Each tree depends only on (seed, t). */
void wl_random_pop(uint64_t seed, int32_t M, const uint64_t *off, uint8_t *buf, int32_t threads)
{
    pop_job j;
    j.seed = seed; j.off = off; j.M = M; j.buf = buf; j.next = 0;
    pthread_mutex_init(&j.mu, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int i = 1; i < threads; i++)
        if (pthread_create(&th[started], NULL, pop_worker, &j) == 0) started++;
    pop_worker(&j);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&j.mu);
}

/* Depth (edges from the root to the deepest leaf) of a prefix tree,
 * used by the generator sanity test against the random-tree depth law. */
int64_t wl_depth(const uint8_t *t, uint64_t n, int64_t *scratch)
{
    /* scratch: per open slot, the depth of the node that fills it */
    int64_t sp = 0, maxd = 0;
    scratch[sp++] = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (sp == 0) return -1;
        int64_t d = scratch[--sp];
        if (d > maxd) maxd = d;
        if (t[i] != WL_X) { scratch[sp++] = d + 1; scratch[sp++] = d + 1; }
    }
    return sp == 0 ? maxd : -1;
}

/* Ephemeral random constants (Sec. 2.1, Table 1): n distinct values drawn at
 * random from the 2001 numbers -1.000, -0.999, ..., +1.000, each the
 * binary32 nearest k/1000 (computed in binary64, rounded once).  A partial
 * Fisher-Yates shuffle of the 2001 indices. */
void wl_erc_table(uint64_t seed, int32_t n, float *out)
{
    int32_t idx[2001];
    for (int32_t i = 0; i < 2001; i++) idx[i] = i - 1000;
    wl_rng r;
    rng_seed(&r, seed, 0xE2C);
    if (n > 2001) n = 2001;
    for (int32_t i = 0; i < n; i++) {
        int32_t j = i + (int32_t)(rng_next(&r) % (uint64_t)(2001 - i));
        int32_t t = idx[i]; idx[i] = idx[j]; idx[j] = t;
        out[i] = (float)((double)idx[i] / 1000.0);
    }
}

/* Leaves of the trees in buf[0, len): each X becomes constant token
 * 6 + j, j uniform over the n_consts constants, with probability 1 - p_x. */
void wl_relabel_leaves(uint64_t seed, uint8_t *buf, uint64_t len, int32_t n_consts, double p_x)
{
    wl_rng r;
    rng_seed(&r, seed, 0x1EAF);
    for (uint64_t i = 0; i < len; i++) {
        if (buf[i] != WL_X || n_consts < 1) continue;
        if (rng_unit(&r) < p_x) continue;
        buf[i] = (uint8_t)(6 + (int32_t)(rng_next(&r) % (uint64_t)n_consts));
    }
}
