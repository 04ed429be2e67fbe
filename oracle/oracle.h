/*
 * Oracle for GP-tree evaluation, fitness, crossover and selection.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, scalar C written from the paper
 * (Langdon & Banzhaf, "Faster Genetic Programming GPquick via multicore and
 * Advanced Vector Extensions", 2019).  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header
 * or constant with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off (no -ffast-math, no FTZ/DAZ).
 *
 * Tokens (one byte per node, root first, Sec. 2.2):
 *   0 ADD, 1 SUB, 2 MUL, 3 DIV (protected), 4 X, and 6 + i for constant i
 *   of a table of up to 250 ephemeral random constants (Sec. 2.1, Table 1).
 * A node "op A B" means A op B: the first argument is evaluated by the first
 * nested EVAL call (Sec. 2.2) and protected division returns
 * (y!=0) ? x/y : 1.0f with x the first argument (Table 1 footnote).
 */
#ifndef GP_ORACLE_H
#define GP_ORACLE_H
#include <stdint.h>

#define OR_ADD 0
#define OR_SUB 1
#define OR_MUL 2
#define OR_DIV 3
#define OR_X 4
/* tokens OR_C0 .. OR_C0 + n_consts - 1: ephemeral random constants (5 is
 * never a valid token of a tree) */
#define OR_C0 6

/* one function node applied to binary32 operands, round-to-nearest-even */
float or_op(int op, float a, float b);

/* 1 if t[0..n) is one complete prefix tree over tokens 0..4, else 0.
 * *max_stack (nullable) receives the largest stack height reached by the
 * right-to-left stack machine of or_eval_cases. */
int or_validate(const uint8_t *t, uint64_t n, uint64_t *max_stack);
/* The same over tokens 0..4 and the n_consts constant tokens. */
int or_validate_c(const uint8_t *t, uint64_t n, int32_t n_consts, uint64_t *max_stack);

/* Value of the tree on each of the N cases x[0..N).  Explicit stack of
 * N-float frames, tokens processed right to left (Sec. 2.2).  Returns 0,
 * or -1 for an invalid tree / allocation failure. */
int or_eval_cases(const uint8_t *t, uint64_t n, const float *x, int32_t N, float *out);
/* The same with constants: token OR_C0 + i pushes consts[i] on every case. */
int or_eval_cases_c(const uint8_t *t, uint64_t n, const float *x, int32_t N, const float *consts,
                    int32_t n_consts, float *out);

/* Mean absolute error, binary32, cases summed in ascending order with a
 * plain loop (Sec. 2.2 last paragraph, Sec. 3.2, Table 1). */
float or_fitness(const float *out, const float *y, int32_t N);

/* Hits (Sec. 3.2, reported only): the cases whose absolute error, the same
 * binary32 term the fitness sums, is at most 0.01 (a NaN error is no hit). */
int32_t or_hits(const float *out, const float *y, int32_t N);

/* Population: fitness[M], per_case[M*N] (nullable).  threads >= 1 assigns
 * trees to threads dynamically (Sec. 2.3); results do not depend on it.
 * Returns 0, or -(t+1) for the first tree t that failed. */
int64_t or_eval_population(const uint8_t *buf, const uint64_t *off, int32_t M,
                           const float *x, const float *y, int32_t N,
                           float *fitness, float *per_case, int32_t threads);
int64_t or_eval_population_c(const uint8_t *buf, const uint64_t *off, int32_t M,
                             const float *x, const float *y, int32_t N, const float *consts,
                             int32_t n_consts, float *fitness, float *per_case, int32_t threads);

/* Depth of a valid tree (edges on its longest root-to-leaf path; a lone
 * leaf has depth 0), or -1 for an invalid tree. */
int64_t or_depth(const uint8_t *t, uint64_t n);

/* End (inclusive) of the subtree rooted at p. */
uint64_t or_subtree_end(const uint8_t *t, uint64_t n, uint64_t p);

/* Subtree crossover (Sec. 3.1): child = mum[0,p) + dad subtree at q +
 * mum after the subtree at p.  Writes the child (if child != NULL) and
 * returns its size. */
uint64_t or_crossover(const uint8_t *mum, uint64_t nm, const uint8_t *dad, uint64_t nd,
                      uint64_t p, uint64_t q, uint8_t *child);

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Selection and crossover points of one child of one generation.
 * mum/dad: tournaments of size k over fitness[M] (lower is better,
 * NaN worst, ties keep the earlier draw); p, q uniform over the parents'
 * nodes. */
void or_choose(const float *fitness, int32_t M, int32_t k, uint64_t seed, uint64_t gen,
               uint32_t child, const uint64_t *sizes, int32_t *mum, int32_t *dad,
               uint64_t *p, uint64_t *q);

/* One generation: M children by tournament + subtree crossover; a child
 * larger than cap is replaced by a copy of its mum.  child_buf must hold
 * cap_bytes; child_off[M+1].  Returns the number of capped children, or -1
 * when child_buf is too small. */
int64_t or_generation(const uint8_t *buf, const uint64_t *off, int32_t M, const float *fitness,
                      int32_t k, uint64_t seed, uint64_t gen, uint64_t size_cap,
                      uint8_t *child_buf, uint64_t cap_bytes, uint64_t *child_off);

#endif
