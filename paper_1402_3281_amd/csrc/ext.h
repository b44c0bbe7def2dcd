// ext.h -- launchers of the Section 4 extension kernels (ext_kernels.hip)
// and the executor steps built on them (ext.hip).
#pragma once

#include "common.h"

namespace sclap {

struct Ctx;
struct Job;
struct Level;

// The graph without the cut edges of a partition blk (n entries): the
// entries (u, v) with blk(u) == blk(v), in their order.  Scratch for m
// entries: filter_tiles(m) tiles of kEpb entries, 32 words per tile.
int64_t filter_tiles(int64_t m);
// kw, wpre: 32 * filter_tiles(m) entries; tcnt: filter_tiles(m) + 1 (the last
// left for the caller to zero).
int filter_mark(const int64_t* rp, const int32_t* col, const int32_t* blk, int64_t n, int64_t m, uint64_t* kw,
                uint32_t* wpre, int64_t* tcnt, const int32_t* trow, hipStream_t st);
// toff: exclusive scan of tcnt (T + 1 entries).
int filter_place(const int32_t* col, const int32_t* ew, int64_t m, const uint64_t* kw, const uint32_t* wpre,
                 const int64_t* toff, int32_t* col2, int32_t* ew2, hipStream_t st);
int filter_rows(const int64_t* rp, int64_t n, int64_t m, const uint64_t* kw, const uint32_t* wpre,
                const int64_t* toff, int64_t T, int64_t* rp2, hipStream_t st);

// bc(cof(v)) = bf(v) for every v with cof(v) >= 0.
int blocks_up(const int32_t* cof, const int32_t* bf, int64_t n, int32_t* bc, hipStream_t st);
// Degree class of every node for S sub-rounds: 0 below degree 4, else
// floor(log4(degree)), at most S - 1.
int degree_classes(const int64_t* rp, int64_t n, int S, uint8_t* cls, hipStream_t st);
// Initial labels of ensemble member e: lab(v) = desire(v) = (a v + b) mod n
// (member_affine), W(lab(v)) = c(v).  Member 0: the node ids.
void member_affine(int64_t n, int32_t e, int64_t* a, int64_t* b);
int init_member(int32_t* lab, int32_t* desire, int64_t* W, const int64_t* nw, int64_t n, int32_t e,
                hipStream_t st);

int overlay_keys(const int32_t* O, const int32_t* C, int64_t n, int bits, uint64_t* keys, int32_t* vals,
                 hipStream_t st);
int overlay_heads(const uint64_t* K, int64_t n, int32_t* head, hipStream_t st);
int overlay_first(const int32_t* V, const int32_t* head, const int32_t* hx, int64_t n, int32_t* segmin,
                  int32_t* first, hipStream_t st);
int overlay_assign(const int32_t* V, const int32_t* head, const int32_t* hx, const int32_t* segmin,
                   const int32_t* rank, int64_t n, int32_t* O, hipStream_t st);

// Executor steps (ext.hip).
// F: the level's graph without the cut edges of blk, sharing L's node
// weights; its own arrays are owned (own_rp, own_col, own_ew).
int build_respect_graph(Ctx* c, const Level& L, const int32_t* blk, Level* F, hipStream_t st);
// Initial labels of ensemble member e >= 1 for the job's current level.
int begin_member_labels(Ctx* c, Job* j, hipStream_t st);
// O := overlay of O and C (n nodes, labels in [0, n)), numbered by first
// occurrence in node order; *count = clusters (may be NULL).
int overlay_labels(Ctx* c, int32_t* O, const int32_t* C, int64_t n, int64_t* count, hipStream_t st);
// L_max on level i of q levels with extra imbalance dnum / dden (Section 4):
// floor((1 + eps + delta / (q - i)) ceil(C / k)) on 1 <= i <= q - 1, lmax on
// level 0 or without delta.
int64_t level_lmax(int64_t C, int32_t k, int64_t eps_num, int64_t eps_den, int64_t dnum, int64_t dden, int32_t q,
                   int32_t i, int64_t lmax);

}  // namespace sclap
