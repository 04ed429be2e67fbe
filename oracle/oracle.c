/*
 * Oracle for GP-tree evaluation - TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written from the paper's description, in the paper's order:
 *   - trees are flattened, root first, one byte per node (Sec. 2.2);
 *   - one pass over the buffer evaluates every test case, keeping an
 *     external stack whose frames hold one float per test case (Sec. 2.2);
 *   - the functions are +, -, x and protected division
 *     (y!=0) ? x/y : 1.0f (Sec. 2.1, Table 1 footnote);
 *   - the terminals are x and up to 250 ephemeral random constants, each a
 *     fixed value the same on every case (Sec. 2.1, Table 1);
 *   - fitness is the mean absolute error over the cases (Table 1, Sec. 3.2),
 *     summed by a plain ascending loop so the order is fixed (Sec. 2.2);
 *   - crossover copies the mum up to the removed subtree, then the dad's
 *     subtree, then the rest of the mum; both points are uniform over all
 *     nodes (Sec. 3.1);
 *   - parents are chosen by tournament (Table 1).
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

float or_op(int op, float a, float b)
{
    switch (op) {
    case OR_ADD: return a + b;
    case OR_SUB: return a - b;
    case OR_MUL: return a * b;
    default:     return (b != 0.0f) ? a / b : 1.0f;
    }
}

/* A leaf: x, or one of the n_consts constants (tokens OR_C0 ..). */
static int is_leaf(uint8_t tok, int32_t n_consts)
{
    return tok == OR_X || (tok >= OR_C0 && tok < OR_C0 + n_consts);
}

int or_validate(const uint8_t *t, uint64_t n, uint64_t *max_stack)
{
    return or_validate_c(t, n, 0, max_stack);
}

int or_validate_c(const uint8_t *t, uint64_t n, int32_t n_consts, uint64_t *max_stack)
{
    /* Open-slot counter: starts at one (the root), each token fills one slot
     * and a function opens two.  The word is one tree iff the counter is
     * positive before every token and zero after the last. */
    int64_t c = 1;
    for (uint64_t i = 0; i < n; i++) {
        if (t[i] >= OR_X && !is_leaf(t[i], n_consts)) return 0;
        if (c < 1) return 0;
        c -= 1;
        if (t[i] < OR_X) c += 2;
    }
    if (n == 0 || c != 0) return 0;
    if (max_stack) {
        /* height of the right-to-left machine: +1 per X, -1 per function */
        int64_t h = 0, m = 0;
        for (uint64_t i = n; i-- > 0;) {
            h += (t[i] < OR_X) ? -1 : 1;
            if (h > m) m = h;
        }
        *max_stack = (uint64_t)m;
    }
    return 1;
}

int or_eval_cases(const uint8_t *t, uint64_t n, const float *x, int32_t N, float *out)
{
    return or_eval_cases_c(t, n, x, N, NULL, 0, out);
}

int or_eval_cases_c(const uint8_t *t, uint64_t n, const float *x, int32_t N, const float *consts,
                    int32_t n_consts, float *out)
{
    uint64_t depth;
    if (!or_validate_c(t, n, n_consts, &depth)) return -1;
    float *stack = (float *)malloc(sizeof(float) * (size_t)depth * (size_t)(N > 0 ? N : 1));
    if (!stack) return -1;
    uint64_t sp = 0; /* number of frames on the stack */
    for (uint64_t k = n; k-- > 0;) {
        uint8_t tok = t[k];
        if (tok == OR_X) {
            float *f = stack + (size_t)sp * (size_t)N;
            for (int32_t i = 0; i < N; i++) f[i] = x[i];
            sp++;
        } else if (tok >= OR_C0) {
            /* an ephemeral random constant: the same value on every case */
            float *f = stack + (size_t)sp * (size_t)N;
            for (int32_t i = 0; i < N; i++) f[i] = consts[tok - OR_C0];
            sp++;
        } else {
            /* top frame = first argument, the frame below = second */
            float *a = stack + (size_t)(sp - 1) * (size_t)N;
            float *b = stack + (size_t)(sp - 2) * (size_t)N;
            for (int32_t i = 0; i < N; i++) b[i] = or_op(tok, a[i], b[i]);
            sp--;
        }
    }
    for (int32_t i = 0; i < N; i++) out[i] = stack[i];
    free(stack);
    return 0;
}

float or_fitness(const float *out, const float *y, int32_t N)
{
    float s = 0.0f;
    for (int32_t i = 0; i < N; i++) s = s + fabsf(out[i] - y[i]);
    return s / (float)N;
}

int32_t or_hits(const float *out, const float *y, int32_t N)
{
    int32_t h = 0;
    for (int32_t i = 0; i < N; i++)
        if (fabsf(out[i] - y[i]) <= 0.01f) h++;
    return h;
}

typedef struct {
    const uint8_t *buf;
    const uint64_t *off;
    int32_t M, N;
    const float *x, *y;
    const float *consts;
    int32_t n_consts;
    float *fitness, *per_case;
    int32_t next;
    int64_t status;
    pthread_mutex_t mu;
} pop_eval;

static void *pop_eval_worker(void *arg)
{
    pop_eval *pe = (pop_eval *)arg;
    float *tmp = (float *)malloc(sizeof(float) * (size_t)(pe->N > 0 ? pe->N : 1));
    for (;;) {
        pthread_mutex_lock(&pe->mu);
        int32_t t = pe->next++;
        pthread_mutex_unlock(&pe->mu);
        if (t >= pe->M) break;
        float *o = pe->per_case ? pe->per_case + (size_t)t * (size_t)pe->N : tmp;
        int rc = tmp ? or_eval_cases_c(pe->buf + pe->off[t], pe->off[t + 1] - pe->off[t], pe->x, pe->N, pe->consts,
                                       pe->n_consts, o)
                     : -1;
        if (rc != 0) {
            pthread_mutex_lock(&pe->mu);
            if (pe->status == 0 || -(pe->status) - 1 > t) pe->status = -(int64_t)t - 1;
            pthread_mutex_unlock(&pe->mu);
            continue;
        }
        pe->fitness[t] = or_fitness(o, pe->y, pe->N);
    }
    free(tmp);
    return NULL;
}

int64_t or_eval_population(const uint8_t *buf, const uint64_t *off, int32_t M,
                           const float *x, const float *y, int32_t N,
                           float *fitness, float *per_case, int32_t threads)
{
    return or_eval_population_c(buf, off, M, x, y, N, NULL, 0, fitness, per_case, threads);
}

int64_t or_eval_population_c(const uint8_t *buf, const uint64_t *off, int32_t M,
                             const float *x, const float *y, int32_t N, const float *consts,
                             int32_t n_consts, float *fitness, float *per_case, int32_t threads)
{
    pop_eval pe;
    pe.buf = buf; pe.off = off; pe.M = M; pe.N = N; pe.x = x; pe.y = y;
    pe.consts = consts; pe.n_consts = n_consts;
    pe.fitness = fitness; pe.per_case = per_case; pe.next = 0; pe.status = 0;
    pthread_mutex_init(&pe.mu, NULL);
    if (threads < 1) threads = 1;
    if (threads > 512) threads = 512;
    pthread_t th[512];
    int started = 0;
    for (int i = 1; i < threads; i++)
        if (pthread_create(&th[started], NULL, pop_eval_worker, &pe) == 0) started++;
    pop_eval_worker(&pe);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&pe.mu);
    return pe.status;
}

int64_t or_depth(const uint8_t *t, uint64_t n)
{
    /* Right to left, as the evaluator reads the tree: a leaf is a subtree of
     * depth 0, a function one more than the deeper of its two arguments
     * (Sec. 4 plots depth against size; the root is at depth 0, as in the
     * ramped half-and-half depths of Table 1). */
    if (!or_validate_c(t, n, 256 - OR_C0, NULL)) return -1;
    int64_t *h = (int64_t *)malloc(sizeof(int64_t) * (size_t)((n + 1) / 2 + 1));
    if (!h) return -1;
    uint64_t sp = 0;
    for (uint64_t k = n; k-- > 0;) {
        if (t[k] >= OR_X) {
            h[sp++] = 0;
        } else {
            int64_t a = h[--sp], b = h[--sp];
            h[sp++] = 1 + (a > b ? a : b);
        }
    }
    int64_t d = h[0];
    free(h);
    return d;
}

uint64_t or_subtree_end(const uint8_t *t, uint64_t n, uint64_t p)
{
    /* the subtree at p is complete once the slots it opened are all filled */
    int64_t open = 1;
    for (uint64_t k = p; k < n; k++) {
        open -= 1;
        if (t[k] < OR_X) open += 2;
        if (open == 0) return k;
    }
    return n - 1; /* not reached for a valid tree */
}

uint64_t or_crossover(const uint8_t *mum, uint64_t nm, const uint8_t *dad, uint64_t nd,
                      uint64_t p, uint64_t q, uint8_t *child)
{
    uint64_t ep = or_subtree_end(mum, nm, p);
    uint64_t eq = or_subtree_end(dad, nd, q);
    uint64_t a = p, b = eq - q + 1, c = nm - (ep + 1);
    if (child) {
        memcpy(child, mum, a);
        memcpy(child + a, dad + q, b);
        memcpy(child + a + b, mum + ep + 1, c);
    }
    return a + b + c;
}

/* ---------------------------------------------------------------- Philox */

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* ------------------------------------------------------------- selection */

/* Draw layout (stated for both implementations):
 *   key = {seed lo32, seed hi32};
 *   ctr = {child, purpose, gen lo32, gen hi32};
 *   tournament candidate c of role r (0 mum, 1 dad) is word c%4 of the
 *   block with purpose ((r+1) << 8) | (c/4), mapped to [0,M) by
 *   (w * M) >> 32;
 *   crossover points use purpose 0x300: p from (w1:w0), q from (w3:w2),
 *   mapped to [0,n) by the high 64 bits of the 128-bit product u * n. */

static int better(float a, float b)
{
    if (isnan(a)) return 0;
    if (isnan(b)) return 1;
    return a < b;
}

static int32_t tournament(const float *fit, int32_t M, int32_t k, const uint32_t key[2],
                          uint64_t gen, uint32_t child, int role)
{
    int32_t best = -1;
    uint32_t w[4];
    for (int32_t c = 0; c < k; c++) {
        if (c % 4 == 0) {
            uint32_t ctr[4] = {child, ((uint32_t)(role + 1) << 8) | (uint32_t)(c / 4),
                               (uint32_t)gen, (uint32_t)(gen >> 32)};
            or_philox4x32_10(ctr, key, w);
        }
        int32_t cand = (int32_t)(((uint64_t)w[c % 4] * (uint64_t)M) >> 32);
        if (best < 0 || better(fit[cand], fit[best])) best = cand;
    }
    return best;
}

static uint64_t mulhi64(uint64_t u, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)u * (unsigned __int128)n) >> 64);
}

void or_choose(const float *fitness, int32_t M, int32_t k, uint64_t seed, uint64_t gen,
               uint32_t child, const uint64_t *sizes, int32_t *mum, int32_t *dad,
               uint64_t *p, uint64_t *q)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int32_t m = tournament(fitness, M, k, key, gen, child, 0);
    int32_t d = tournament(fitness, M, k, key, gen, child, 1);
    uint32_t ctr[4] = {child, 0x300u, (uint32_t)gen, (uint32_t)(gen >> 32)};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    uint64_t up = ((uint64_t)w[1] << 32) | w[0];
    uint64_t uq = ((uint64_t)w[3] << 32) | w[2];
    *mum = m;
    *dad = d;
    *p = mulhi64(up, sizes[m]);
    *q = mulhi64(uq, sizes[d]);
}

int64_t or_generation(const uint8_t *buf, const uint64_t *off, int32_t M, const float *fitness,
                      int32_t k, uint64_t seed, uint64_t gen, uint64_t size_cap,
                      uint8_t *child_buf, uint64_t cap_bytes, uint64_t *child_off)
{
    uint64_t *sizes = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)M);
    if (!sizes) return -1;
    for (int32_t i = 0; i < M; i++) sizes[i] = off[i + 1] - off[i];
    int64_t capped = 0;
    child_off[0] = 0;
    for (int32_t j = 0; j < M; j++) {
        int32_t m, d;
        uint64_t p, q;
        or_choose(fitness, M, k, seed, gen, (uint32_t)j, sizes, &m, &d, &p, &q);
        const uint8_t *mt = buf + off[m], *dt = buf + off[d];
        uint64_t n = or_crossover(mt, sizes[m], dt, sizes[d], p, q, NULL);
        uint64_t at = child_off[j];
        if (n > size_cap) {
            capped++;
            n = sizes[m];
            if (at + n > cap_bytes) { free(sizes); return -1; }
            memcpy(child_buf + at, mt, n);
        } else {
            if (at + n > cap_bytes) { free(sizes); return -1; }
            or_crossover(mt, sizes[m], dt, sizes[d], p, q, child_buf + at);
        }
        child_off[j + 1] = at + n;
    }
    free(sizes);
    return capped;
}
