/*
 * CPU oracle for the contig-generation path (Guidi et al., "Distributed-Memory
 * Parallel Contig Generation for De Novo Long-Read Genome Assembly", ICPP'22,
 * Algorithm 2 and Sections 4.2-4.4).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded reference
 * that the parity tests, the smoke check and the benchmark's CPU baseline call
 * to decide what the GPU library must produce.  The GPU library never links,
 * loads or calls it, and it shares no code, header or table with the GPU
 * library.
 *
 * All arrays are host arrays owned by the caller.  Vertex ids are 0-based.
 * Graph input format: symmetric CSR (row_ptr[n+1], col[m]), per entry an
 * overlap length ovl[m] and strand bits strand[m] (bit0 s: the source read is
 * reverse-complemented when the walk leaves it along this entry; bit1 d: the
 * destination read is reverse-complemented when the walk enters it), read
 * lengths, 16-aligned base offsets, and a 2-bit packed base store (16 bases
 * per 32-bit word, base i at bits 2*(i%16), A=0 C=1 G=2 T=3).
 */
#ifndef CGORACLE_H
#define CGORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CGO_SINGLE = 0, CGO_PATH = 1, CGO_CYCLE = 2 };
enum { CGO_CIRCULAR = 1, CGO_SAME_END_JOIN = 2, CGO_SINGLE_READ = 4 };

/* Input checks (string matrix symmetric, twin strand bits, overlap bounds,
 * and, when given, pre/post inside their reads).
 * Returns -1 when valid, else the index of the first offending entry (or
 * vertex, or -2 for a bad row_ptr frame); *why receives a reason code. */
int64_t cgo_validate(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col,
                     const uint32_t *ovl, const uint8_t *strand, const uint32_t *read_len,
                     const uint64_t *read_off, uint64_t seq_words, const uint32_t *pre,
                     const uint32_t *post, int32_t *why);

/* Branch removal (Section 4.2): degree = nonzeros in the row; branch <=>
 * degree >= 3; an entry survives in L iff neither endpoint is a branch.
 * flags[v]: bit0 branch, bit1/bit2 entry 0/1 of row v kept.
 * counts[0] = branch vertices, counts[1] = kept directed entries. */
void cgo_mask(int32_t n, const int32_t *row_ptr, const int32_t *col, uint8_t *flags,
              int32_t *counts);

/* Connected components of L (Section 4.2) by union-find; each vertex gets the
 * smallest vertex id of its component. */
void cgo_components(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint8_t *flags,
                    int32_t *label);

/* Component table: size q (reads), kind (single / path / cycle), eligible
 * components (not a branch vertex, q >= min_reads) in ascending label order.
 * label_comp[r] = index of the eligible component labelled r, else -1.
 * Returns the number of eligible components, or -1 if a component is neither
 * a path nor a cycle (impossible for degree <= 2). */
int32_t cgo_table(int32_t n, const int32_t *row_ptr, const uint8_t *flags, const int32_t *label,
                  int32_t min_reads, int32_t *comp_label, int32_t *comp_size, uint8_t *comp_kind,
                  int32_t *label_comp);

/* Greedy multiway number partitioning, LPT (Section 4.3): component weights
 * (the read counts, or any other weights) sorted in decreasing order (ties
 * by ascending label), each to the least loaded of P bins (ties by lowest
 * bin index); bin_load[b] = sum of the weights in bin b. */
void cgo_lpt(int32_t n_comp, const uint64_t *weight, const int32_t *comp_label, int32_t P,
             int32_t *comp_bin, uint64_t *bin_load);

/* Order of the components by (bin, label): comp_rank[c] is c's position in
 * that order and comp_start[c] the number of reads of the components before
 * it, i.e. where c's reads start in the induced local numbering. */
void cgo_order(int32_t n_comp, const int32_t *comp_label, const int32_t *comp_bin,
               const int32_t *comp_size, int32_t *comp_rank, int32_t *comp_start);

/* Induced subgraph (Section 4.3): eligible vertices renumbered by
 * (bin, label, id); local CSR of their kept entries in original row order,
 * columns mapped to local numbers, original entry index kept.
 * bin_vptr[b] = reads of the bins before b (counted from comp_size).
 * sizes[0] = n_e (local vertices), sizes[1] = m_e (local entries). */
void cgo_induce(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint8_t *flags,
                const int32_t *label, int32_t n_comp, const int32_t *label_comp,
                const int32_t *comp_bin, const int32_t *comp_start, int32_t P,
                const int32_t *comp_size, int32_t *perm, int32_t *bin_vptr,
                int32_t *loc_row_ptr, int32_t *loc_col, int32_t *loc_eid, int32_t *sizes);

/* Local assembly (Section 4.4): for every eligible component in (bin, label)
 * order, walk its chain from the start root and concatenate the read pieces
 * l_r[alpha:pre(e0)] + l_c1[post(e0):pre(e1)] + ... + l_r'[post(e_{q-2}):beta].
 * pre / post (per entry, stored coordinates) may be NULL: then they follow
 * from the overlap lengths.  A piece whose end lies before its start is
 * empty.  Contig k (in (bin, label) order) is written 2-bit packed at base offset
 * rec_base_off[k] (exclusive prefix of 16*ceil(len/16)); padding bits are 0.
 * Returns 0, or -4 when the contigs need more than cap_words words (then only
 * *total_words and the records are written). */
int32_t cgo_assemble(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *ovl,
                     const uint8_t *strand, const uint32_t *read_len, const uint64_t *read_off,
                     const uint32_t *seq, const uint32_t *pre, const uint32_t *post,
                     int32_t n_comp, const int32_t *comp_label,
                     const int32_t *comp_size, const uint8_t *comp_kind, const int32_t *comp_bin,
                     const int32_t *comp_rank, const int32_t *comp_start, const int32_t *perm,
                     const int32_t *loc_row_ptr, const int32_t *loc_col, const int32_t *loc_eid,
                     int32_t *rec_label, int32_t *rec_bin, int32_t *rec_start,
                     int32_t *rec_nreads, uint64_t *rec_len, uint64_t *rec_base_off,
                     uint32_t *rec_flags, int32_t *rec_layout_off, int32_t *layout_vid,
                     uint8_t *layout_rev, uint32_t *bases, uint64_t cap_words,
                     uint64_t *total_words);

/* The step before the path (Algorithm 1: Prune(IsContainedRead), then
 * TransitiveReduction; Section 2's string-graph definitions), on an overlap
 * graph R given like S (symmetric CSR, overlap length and strand bits per
 * entry):
 *   contained[v] = 1 when some entry u->v covers all of v (ovl >= len(v))
 *                  and u is longer than v, or as long with a smaller id
 *                  (reading: of identical reads the smallest id stays);
 *   an entry u->w between reads that are not contained is transitive when a
 *   third read v, not contained, has entries u->v and v->w that make a valid
 *   walk u, v, w with the same end orientations as u->w (s(u->v) = s(u->w),
 *   d(u->v) = s(v->w), d(v->w) = d(u->w)) and whose overhangs add up to that
 *   of u->w within fuzz: |sfx(u->v) + sfx(v->w) - sfx(u->w)| <= fuzz, with
 *   sfx(x->y) = len(y) - ovl(x->y) (reading: a parallel path of two edges
 *   carrying the same information);
 *   the pair {u, w} leaves S when either of its entries is transitive or
 *   either read is contained.
 * kept[e] = 1 for the entries of R that stay; S keeps R's column order
 * (s_row_ptr[n+1], s_col / s_ovl / s_strand of up to row_ptr[n] entries).
 * Returns the number of entries of S. */
int64_t cgo_reduce(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *ovl,
                   const uint8_t *strand, const uint32_t *read_len, uint32_t fuzz,
                   uint8_t *contained, uint8_t *kept, int32_t *s_row_ptr, int32_t *s_col,
                   uint32_t *s_ovl, uint8_t *s_strand);

#ifdef __cplusplus
}
#endif
#endif
