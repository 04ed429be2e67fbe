// Host-side launchers of the libev kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "ev_internal.h"

namespace ev {
// Launchers taking a GLevel* (gl, nullable) serve a plan made on the device
// too: the count arguments are then the capacities the grid is launched
// for, and the kernels take the live counts from gl.
hipError_t launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t s);
// n bytes, by a kernel on s (one end may be pinned host memory)
hipError_t launch_copy(void* dst, const void* src, uint64_t n, hipStream_t s);
hipError_t launch_seg_build(const ChunkIn* ch, const ChunkSegs* cg, uint32_t n, uint32_t seg_len, uint32_t head,
                            SegIn* seg, hipStream_t s, const GLevel* gl = nullptr);
hipError_t launch_plan_chunks(const TreeLvl* trees, uint32_t n_trees, uint32_t seg_len, uint32_t head, ChunkIn* ch,
                              ChunkSegs* cg, uint32_t* err_init, uint32_t n_err, hipStream_t s,
                              const GLevel* gl = nullptr);
hipError_t launch_plan_bases(const TreeLvl* trees, uint32_t n_trees, const TreeSum* sum, TreeBase* base, hipStream_t s,
                             const GLevel* gl = nullptr);
hipError_t launch_plan_trees(const TreeLvl* trees, uint32_t n_trees, const ChunkStat* cs, uint32_t level,
                             uint64_t prev_out, uint64_t* code_loc, uint64_t* out_loc, uint64_t* frag_loc,
                             uint32_t* in_end, TreeSum* sum, hipStream_t s, const GLevel* gl = nullptr);
hipError_t launch_plan_items(const ChunkIn* ch, uint32_t n, const TreeBase* base, const uint64_t* code_loc,
                             const uint64_t* out_loc, const uint64_t* frag_loc, const uint32_t* in_end,
                             const uint32_t* cursor,
                             uint64_t* code_begin, uint64_t* frag_end, RunChunk* run, EvalChunk* slow,
                             uint32_t* code_tail, uint8_t* frag_tail, hipStream_t s, const GLevel* gl = nullptr,
                             uint32_t* item_tree = nullptr);
// children reusing their mum's level-0 chunks
hipError_t launch_reuse_runs(const XoPlan* plan, const int32_t* mum, const L0Tree* trees, const ChunkIn* mum_ch,
                             uint32_t n, ReuseRun* out, hipStream_t s);
hipError_t launch_reuse_chunks(const TreeReuse* trees, uint32_t n_trees, const ChunkIn* mum_ch, uint32_t seg_len,
                               uint32_t head, ChunkIn* ch, ChunkSegs* cg, uint32_t* src, uint32_t* err_init,
                               uint32_t n_err, hipStream_t s);
hipError_t launch_reuse_stats(const uint32_t* src, uint32_t n, const ChunkStat* mum_stat, ChunkStat* cstat,
                              hipStream_t s);
hipError_t launch_reuse_copy(const uint32_t* src, uint32_t n, const ChunkStat* cstat, const uint64_t* code_begin,
                             const uint64_t* frag_end, const uint64_t* mum_code, const uint64_t* mum_frag,
                             const uint32_t* mum_codes, const uint8_t* mum_skel, uint32_t* codes, uint8_t* skel,
                             hipStream_t s);
// population statistics: best fitness and convergence, sizes; trees' stack
// heights (bounds for the depth pass's stacks) and depths
hipError_t launch_pop_stats(const float* fit, const uint64_t* off, uint32_t M, PopStatsDev* out, hipStream_t s);
hipError_t launch_tree_height(const uint8_t* buf, const uint64_t* off, uint32_t M, uint32_t* height, hipStream_t s);
hipError_t launch_tree_depth(const uint8_t* buf, const uint64_t* off, uint32_t M, const uint64_t* base, uint32_t* stack,
                             uint32_t* depth, hipStream_t s);
// ref_ok: REF tokens belong to the level's alphabet; n_consts constant tokens do
hipError_t launch_seg_fn(const uint8_t* seq, const SegIn* segs, uint32_t n, SegFn* out, uint32_t ref_ok,
                         uint32_t n_consts, hipStream_t s, const GLevel* gl = nullptr);
hipError_t launch_seg_scan(const ChunkSegs* cseg, uint32_t n, const SegFn* fn, SegStart* st, ChunkStat* cstat,
                           hipStream_t s, const GLevel* gl = nullptr);
// rk/rf/rec (nullable): record the segments' code kinds and fragment tokens
hipError_t launch_seg_count(const uint8_t* seq, const SegIn* segs, uint32_t n, const SegStart* st, SegCount* out,
                            uint8_t* rk, uint8_t* rf, SegRec* rec, uint32_t* ovf, uint32_t seg_len, hipStream_t s,
                            const GLevel* gl = nullptr);
// places recorded segments and validates their codes (as launch_seg_check)
hipError_t launch_seg_place(const SegIn* segs, uint32_t n, const SegCount* cnt, const SegRec* rec, const SegStart* st,
                            const uint64_t* seg_code, const uint64_t* seg_frag, const uint8_t* rk, const uint8_t* rf,
                            uint32_t* codes, uint64_t n_codes, uint8_t* dst, uint64_t n_frag, uint32_t slab_entries,
                            uint32_t* err, uint32_t seg_len, hipStream_t s, const GLevel* gl = nullptr);
hipError_t launch_seg_chunk(const ChunkSegs* cseg, uint32_t n, const SegCount* cnt, ChunkStat* cstat,
                            const uint64_t* code_begin, const uint64_t* frag_end, uint64_t* seg_code, uint64_t* seg_frag,
                            hipStream_t s, const GLevel* gl = nullptr);
hipError_t launch_seg_emit(const uint8_t* seq, const SegIn* segs, uint32_t n, const SegStart* st, const uint64_t* seg_code,
                           const uint64_t* seg_frag, uint8_t* dst, uint32_t* codes, hipStream_t s,
                           const GLevel* gl = nullptr);
hipError_t launch_seg_check(const uint32_t* codes, const SegIn* segs, uint32_t n, const SegStart* st,
                            const uint64_t* seg_code, const SegCount* cnt, uint32_t slab_entries, uint32_t* err,
                            hipStream_t s, const GLevel* gl = nullptr);
size_t eval_lds_bytes(int D);
hipError_t eval_occupancy(int D, int* blocks_per_cu);
hipError_t launch_eval(int D, const EvalArgs& a, uint32_t grid, hipStream_t s);
hipError_t run_occupancy(int* blocks_per_cu);
hipError_t launch_run(const RunArgs& a, uint32_t grid, hipStream_t s);
// the skeleton levels of a plan in one launch (see k_run_chain)
hipError_t chain_occupancy(int* blocks_per_cu);
hipError_t launch_run_chain(const ChainArgs& a, uint32_t grid, hipStream_t s);


hipError_t launch_fitness(const FitArgs& a, hipStream_t s);
hipError_t launch_subtree_end(const uint8_t* buf, const uint64_t* base, const uint64_t* pos, uint32_t n,
                              uint64_t* end_out, hipStream_t s);
hipError_t launch_xo_copy(const uint8_t* mums, const uint8_t* dads, const XoPlan* plan, const uint64_t* off,
                          uint32_t n, uint64_t pieces, uint8_t* dst, uint8_t* pad, uint32_t pad_len, hipStream_t s,
                          const uint32_t* stop = nullptr);
hipError_t launch_xo_query(const uint64_t* moff, const uint64_t* doff, const int32_t* mum, const int32_t* dad,
                           const uint64_t* p, const uint64_t* q, uint32_t n, uint64_t* qb, uint64_t* qp, hipStream_t s);
hipError_t launch_xo_plan(const uint64_t* moff, const uint64_t* doff, const int32_t* mum, const int32_t* dad,
                          const uint64_t* p, const uint64_t* q, const uint64_t* ends, uint32_t n, uint64_t cap,
                          XoPlan* plan, uint64_t* off, hipStream_t s, const uint64_t* mlen = nullptr);
// a batch of children to places of their own (see k_xo_copy_at)
hipError_t launch_xo_copy_at(const uint8_t* src, const XoPlan* plan, const uint32_t* idx, const uint64_t* at,
                             const uint64_t* pf, uint32_t n, uint64_t pieces, uint8_t* dst, hipStream_t s);
hipError_t launch_select(const float* fit, const uint64_t* off, uint32_t M, int32_t k, uint64_t seed, uint64_t gen,
                         int32_t* mum, int32_t* dad, uint64_t* p, uint64_t* q, hipStream_t s,
                         const uint64_t* gen_at = nullptr, const uint64_t* len = nullptr);
// a generation replayed from a graph: the children's trees, each plan
// level's first and last step, and the generation's verdict
hipError_t launch_g_init(const uint64_t* off, uint32_t M, GTree* tr, uint64_t bytes_cap, uint32_t pad_len,
                         uint64_t pieces_cap, GStatus* st, uint32_t* counters, uint32_t n_counters, hipStream_t s);
hipError_t launch_g_begin(const GTree* tr, uint32_t M, GLevel* gls, uint32_t level, const GCap* caps, uint64_t C,
                          uint32_t seg_len, uint32_t head, uint32_t record, TreeLvl* tl, uint32_t* bucket_start,
                          GStatus* st, hipStream_t s);
hipError_t launch_g_end(GTree* tr, GLevel* gls, uint32_t level, const GCap* caps, uint32_t n_levels, const TreeLvl* tl,
                        const TreeSum* sum, TreeBase* tb, uint32_t* fin, GStatus* st, hipStream_t s);
hipError_t launch_g_finish(GStatus* st, const GLevel* gls, uint32_t n_levels, const uint32_t* err, const float* fit,
                           uint32_t M, uint64_t* gen_at, GStatus* h_st, GLevel* h_levels, float* h_fit, hipStream_t s);
}  // namespace ev
