/*
 * cg.h -- C ABI of the MI355X (gfx950) contig-generation library (libcg).
 *
 * The library implements the contig-generation step of long-read assembly
 * described by Guidi et al., "Distributed-Memory Parallel Contig Generation
 * for De Novo Long-Read Genome Assembly" (ICPP'22), Algorithm 2
 * (ContigGeneration): BranchRemoval -> ConnectedComponent ->
 * GreedyPartitioning -> InducedSubgraph -> LocalAssembly.  Each of those five
 * steps is one call below; every step runs in hand-written HIP kernels on one
 * GPU.
 *
 * Conventions shared by every call
 * --------------------------------
 * * Pointers inside the structs and the array arguments are DEVICE pointers
 *   unless marked [host].  The caller allocates and owns every buffer; the
 *   library never frees or resizes caller memory.
 * * `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *   enqueues work on `stream` and returns; outputs are valid once the stream
 *   has completed.  No call synchronises the host, so the sequence can be
 *   captured into a HIP graph.
 * * Return value: CG_OK (0) or a negative error code.  Argument errors are
 *   detected on the host before anything is enqueued.  Conditions that only
 *   the device can see (an output capacity too small) are reported through
 *   device-side counts that the caller reads after the stream completes, and
 *   through cg_ctx_status().
 * * Only cg_validate() inspects the graph's contents.  The other calls
 *   require a graph that passes it: they follow the graph's indices, so on an
 *   invalid graph both their outputs and their memory accesses are undefined.
 *   Run cg_validate on any graph that does not come from a trusted producer.
 * * A cg_ctx owns a device scratch area and must be used by one host thread
 *   and one stream at a time; independent contexts may share a device.
 * * No C++ exception crosses this interface.
 */
#ifndef CG_H
#define CG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CG_OK            0
#define CG_EINVAL       -1  /* bad argument, shape or pointer                    */
#define CG_ENOMEM       -2  /* context scratch smaller than cg_footprint() states */
#define CG_EHIP         -3  /* HIP runtime error; text in cg_last_error()         */
#define CG_ECAPACITY    -4  /* a device-side count exceeded a caller capacity     */
#define CG_EUNSUPPORTED -5  /* valid request outside the library's limits         */

/* ---- component kinds and contig flags ---------------------------------- */
#define CG_KIND_SINGLE 0    /* one read, no kept edge                              */
#define CG_KIND_PATH   1    /* q reads, q-1 edges: two roots of degree 1           */
#define CG_KIND_CYCLE  2    /* q reads, q edges: every read has degree 2           */

#define CG_CONTIG_CIRCULAR      1u  /* cycle cut before its smallest read           */
#define CG_CONTIG_SAME_END_JOIN 2u  /* a read is entered and left on the same end   */
#define CG_CONTIG_SINGLE        4u  /* one-read contig (only when min_reads <= 1)   */

/* device status bits reported by cg_ctx_status() */
#define CG_STATUS_BASES_OVERFLOW 1u /* cg_assemble: contigs need more than cap_words */
#define CG_STATUS_SCAN_STALLED   2u /* a scan stopped waiting for a block that never
                                       published (results of that call are invalid) */
#define CG_STATUS_WEIGHT_RANGE   4u /* cg_partition: a bases weight of 2^32 or more */

/*
 * The string graph S (Section 2: a bidirected graph, stored as a symmetric
 * sparse matrix; Section 4.2 calls it the string matrix).
 *   n, m      vertices (= reads, ids 0..n-1) and directed entries; 0 <= n < 2^30,
 *             0 <= m < 2^31.
 *   row_ptr   int32[n+1], col int32[m]: CSR of S, columns strictly increasing
 *             inside a row, no self loops; entry (u,v) present iff (v,u) is.
 *   ovl       uint32[m]: overlap length of reads u and v, equal in both
 *             directions, 1 <= ovl < min(read_len[u], read_len[v]).
 *   strand    uint8[m]: bit0 s = read u is reverse-complemented when the walk
 *             leaves u along this entry; bit1 d = read v is reverse-complemented
 *             when the walk enters v along it.  The twin entry (v,u) carries
 *             (s', d') = (!d, !s).  Other bits are zero.
 *   read_len  uint32[n], >= 1.
 *   read_off  uint64[n]: base offset of read v in seq, a multiple of 16.
 *   seq       uint32[seq_words]: 2-bit packed bases, 16 per word, base i of the
 *             store at bits 2*(i%16) of word i/16; A=0 C=1 G=2 T=3, so the
 *             complement of a base is x^3.
 *   pre, post optional uint32[m] each (both NULL or both set): the per-entry
 *             values of Section 4.4, in the stored coordinates of each read.
 *             For entry e = (u,v), pre[e] is the last base of read u before
 *             its overlap with v and post[e] the first base of read v inside
 *             it, both in the direction the walk takes the read (increasing
 *             for a forward read, decreasing for a reverse-complemented one).
 *             They carry alignment overhangs (an x-drop alignment may stop
 *             short of a read's end).  With both NULL they follow from ovl:
 *             pre = len(u)-ovl-1 or ovl, post = 0 or len(v)-1.  A read's
 *             piece runs from post of the entry it is entered by to pre of
 *             the entry it leaves by (its whole first / last part for the
 *             walk's first / last read); a piece whose end falls before its
 *             start is empty.  cg_validate checks pre[e] < read_len[u] and
 *             post[e] < read_len[v].
 */
typedef struct {
  int32_t n;
  int32_t m;
  const int32_t  *row_ptr;
  const int32_t  *col;
  const uint32_t *ovl;
  const uint8_t  *strand;
  const uint32_t *read_len;
  const uint64_t *read_off;
  const uint32_t *seq;
  uint64_t seq_words;
  const uint32_t *pre;
  const uint32_t *post;
} cg_graph;

/*
 * Components and their partition (Sections 4.2 and 4.3).  Component arrays
 * hold the ELIGIBLE components (not a branch vertex, at least min_reads
 * reads) in ascending label order; capacity n each, the first *d_n_comp are
 * valid.
 *   comp_label  smallest vertex id of the component
 *   comp_size   q = number of reads
 *   comp_kind   CG_KIND_*
 *   comp_bin    bin (process) chosen by LPT, 0..P-1
 *   comp_rank   position of the component in (bin, label) order
 *   comp_start  number of reads of the components before it in that order
 *   bin_load    uint64[P]: reads per bin
 *   label_comp  int32[n]: for vertex id r, the index of the eligible
 *               component labelled r, else -1
 *   d_n_comp    int32[1]
 */
typedef struct {
  int32_t  *comp_label;
  int32_t  *comp_size;
  uint8_t  *comp_kind;
  int32_t  *comp_bin;
  int32_t  *comp_rank;
  int32_t  *comp_start;
  uint64_t *bin_load;
  int32_t  *label_comp;
  int32_t  *d_n_comp;
} cg_parts;

/*
 * Induced subgraphs of all bins in one local numbering (Section 4.3,
 * InducedSubgraph): local vertex i is read perm[i]; vertices are numbered by
 * (bin, label, id), so bin b owns local vertices bin_vptr[b] ..
 * bin_vptr[b+1]-1 and each component a contiguous block.  Row i of the local
 * CSR lists the kept entries of read perm[i] in the row order of S, with the
 * column renumbered locally (loc_col) and the entry's index in S (loc_eid).
 *   perm int32[n], bin_vptr int32[P+1], loc_row_ptr int32[n+1],
 *   loc_col int32[2n], loc_eid int32[2n], d_sizes int32[2] = (n_e, m_e).
 */
typedef struct {
  int32_t *perm;
  int32_t *bin_vptr;
  int32_t *loc_row_ptr;
  int32_t *loc_col;
  int32_t *loc_eid;
  int32_t *d_sizes;
} cg_local;

/*
 * Contigs (Section 4.4, LocalAssembly): one record per eligible component,
 * records in (bin, label) order (record k belongs to the component with
 * comp_rank == k).  Record arrays have capacity n.
 *   label, bin      of the component
 *   start           read the walk starts from
 *   n_reads         q
 *   len             bases in the contig
 *   base_off        base offset of the contig in `bases` (multiple of 16)
 *   cflags          CG_CONTIG_*
 *   layout_off      first layout entry of the contig (= its comp_start)
 *   layout_vid      int32[n]: reads in walk order
 *   layout_rev      uint8[n]: 1 if that read is reverse-complemented
 *   bases           uint32[cap_words]: contigs 2-bit packed like seq, each
 *                   starting on a word boundary, padding bits zero
 *   d_total_words   uint64[1]: words the contigs need; when it exceeds
 *                   cap_words nothing is written to `bases` and
 *                   CG_STATUS_BASES_OVERFLOW is raised.  cap_words =
 *                   seq_words always suffices.
 */
typedef struct {
  int32_t  *label;
  int32_t  *bin;
  int32_t  *start;
  int32_t  *n_reads;
  uint64_t *len;
  uint64_t *base_off;
  uint32_t *cflags;
  int32_t  *layout_off;
  int32_t  *layout_vid;
  uint8_t  *layout_rev;
  uint32_t *bases;
  uint64_t  cap_words;
  uint64_t *d_total_words;
} cg_contigs;

typedef struct cg_ctx cg_ctx;

/* ---- context ----------------------------------------------------------- */

/* Create a context on `device` with a device scratch area of scratch_bytes
 * (see cg_footprint).  *out receives the context.  Errors: CG_EINVAL (bad
 * device or NULL out), CG_EHIP. */
int cg_ctx_create(int device, size_t scratch_bytes, cg_ctx **out);

/* Release the context and its scratch.  The caller must make sure no work
 * that uses it is still in flight. */
int cg_ctx_destroy(cg_ctx *ctx);

/* Device bytes of one graph of n reads, m directed entries, seq_words
 * packed words and P bins (the signature of Algorithm 2: the string graph S
 * and the read sequences, Section 4.1), for sizing a context and for
 * admitting work by its HBM footprint.  All figures are exact sums of the
 * buffer sizes this header states; allocator rounding is the caller's.
 *   scratch  the context scratch the five calls need (cg_ctx_create)
 *   graph    the cg_graph arrays: row_ptr (n+1), col, ovl, strand (m each),
 *            read_len, read_off (n each), seq (seq_words), and pre, post (m
 *            each) when coords is nonzero
 *   outputs  every output buffer of the five calls at the capacities stated
 *            below (n per record array, 2n local entries, P bins), with
 *            cap_words = seq_words for the packed contigs
 * out is [host].  Errors: CG_EINVAL for a NULL out, negative n, m or
 * seq_words beyond 2^62, or P outside [1, 65536]. */
typedef struct {
  uint64_t scratch;
  uint64_t graph;
  uint64_t outputs;
} cg_sizes;
int cg_footprint(int32_t n, int32_t m, uint64_t seq_words, int32_t P, int32_t coords,
                 cg_sizes *out);

/* Device status bits (CG_STATUS_*) raised since the last clear.  Waits for
 * `stream`, then copies the word to *status [host]; clears it if `clear`. */
int cg_ctx_status(cg_ctx *ctx, void *stream, uint32_t *status, int clear);

/* Per-kernel timing (benchmarks): with max_launches > 0 every kernel launch
 * of the library, up to max_launches of them, is bracketed by two HIP events
 * recorded on the stream it is launched on; 0 switches timing off.  Recording
 * events adds a little time between kernels. */
int cg_ctx_profile(cg_ctx *ctx, int32_t max_launches);

/* Waits for the recorded events and reports, per kernel name, the number of
 * launches and their summed duration in ms, then clears the record.  names,
 * launches and ms are [host] arrays of `cap` entries; names[i] point to
 * static strings; *n_kernels [host] receives the count, *dropped [host,
 * optional] the launches that found no free event pair. */
int cg_ctx_profile_read(cg_ctx *ctx, int32_t cap, const char **names, int64_t *launches,
                        double *ms, int32_t *n_kernels, int64_t *dropped);

/* ---- before the path: an overlap graph reduced to a string graph ------- */

/* Prune(IsContainedRead) and TransitiveReduction (Algorithm 1; Section 2
 * defines redundant vertices and redundant edges) of an overlap graph r,
 * given like a string graph (symmetric CSR with overlap lengths and strand
 * bits, and read lengths; sequences and pre/post are not read):
 *   contained[v] = 1 when an entry u->v covers all of v (ovl >= len(v)) and
 *   u is longer than v, or as long with a smaller id;
 *   an entry u->w between reads that are not contained is transitive when a
 *   third read v, not contained, gives a valid walk u, v, w with u->w's end
 *   orientations (s(u->v) = s(u->w), d(u->v) = s(v->w), d(v->w) = d(u->w))
 *   whose overhangs sfx(x->y) = len(y) - ovl(x->y) add up to u->w's within
 *   `fuzz` bases;
 *   a pair leaves the string graph when either of its entries is transitive
 *   or either read is contained.
 * Outputs [device, caller-owned]: contained u8[n]; kept u8[r->m], 1 for the
 * entries of r that stay; the string graph as s_row_ptr i32[n+1], s_col
 * i32[r->m], s_ovl u32[r->m], s_strand u8[r->m] (r's column order within a
 * row; contained reads keep their ids with empty rows); d_m i32[1] its entry
 * count.  Needs a context sized for (r->n, r->m, 1).  Errors: CG_EINVAL for
 * NULL arguments or a malformed frame, CG_ENOMEM for a small context. */
int cg_reduce(cg_ctx *ctx, const cg_graph *r, uint32_t fuzz, uint8_t *contained, uint8_t *kept,
              int32_t *s_row_ptr, int32_t *s_col, uint32_t *s_ovl, uint8_t *s_strand,
              int32_t *d_m, void *stream);

/* Thread-local text of the last error. */
const char *cg_last_error(void);

/* ---- the five steps of Algorithm 2 ------------------------------------- */

/* Input checks: row_ptr frame and monotonicity, read length >= 1, read
 * offsets 16-aligned and inside seq, column range, no self loop, strictly
 * increasing columns, twin entry present with equal ovl and strand bits
 * (!d, !s), 1 <= ovl < min read length.  d_bad int64[2] receives (index, why)
 * of the first failure in the order just listed ((-1, 0) when valid; index
 * -2 for a bad frame).  why: 1 frame/monotone, 2 column range, 3 self loop,
 * 4 order/duplicate, 5 missing twin, 6 twin ovl, 7 twin strand bits,
 * 8 ovl bounds, 9 read_len, 10 read_off alignment, 11 read past seq. */
int cg_validate(cg_ctx *ctx, const cg_graph *g, int64_t *d_bad, void *stream);

/* BranchRemoval(S) -> L (Section 4.2).  The degree of a vertex is the number
 * of entries in its row; a branch vertex has degree >= 3.  L keeps the
 * entries of S whose two ends are not branch vertices, in place (same
 * indexing).  flags uint8[n]: bit0 = branch, bit1 / bit2 = entry 0 / 1 of the
 * row is kept (only rows of degree <= 2 keep entries).  d_counts int32[2] =
 * (branch vertices, kept directed entries). */
int cg_mask_branches(cg_ctx *ctx, const cg_graph *g, uint8_t *flags, int32_t *d_counts,
                     void *stream);

/* ConnectedComponent(L) -> v (Section 4.2).  label int32[n]: the smallest
 * vertex id of the vertex's component in L (branch and isolated vertices
 * label themselves). */
int cg_components(cg_ctx *ctx, const cg_graph *g, const uint8_t *flags, int32_t *label,
                  void *stream);

/* Contig sizes and GreedyPartitioning(v, P) -> p (Sections 4.2 and 4.3):
 * component sizes and kinds, eligible components (min_reads <= 1 is taken
 * as 1), then LPT: weights in decreasing order (ties: ascending label), each
 * to the least loaded of the P bins (ties: lowest bin index).  Fills `out`
 * (cg_parts above; bin_load holds the sum of the bin's weights).
 * 1 <= P <= 65536.
 *   weight  CG_WEIGHT_READS: a component weighs its read count, the size the
 *           paper partitions by (Section 4.3); CG_WEIGHT_BASES: the total
 *           length of its reads, the work of assembling it.  Bases weights
 *           must stay below 2^32 per component; a larger one raises
 *           CG_STATUS_WEIGHT_RANGE and leaves the partition invalid. */
#define CG_WEIGHT_READS 0
#define CG_WEIGHT_BASES 1
int cg_partition(cg_ctx *ctx, const cg_graph *g, const uint8_t *flags, const int32_t *label,
                 int32_t P, int32_t min_reads, int32_t weight, const cg_parts *out,
                 void *stream);

/* InducedSubgraph(L, p) (Section 4.3): the bins' induced subgraphs in one
 * local numbering; fills `out` (cg_local above). */
int cg_induce(cg_ctx *ctx, const cg_graph *g, const uint8_t *flags, const int32_t *label,
              const cg_parts *parts, int32_t P, const cg_local *out, void *stream);

/* LocalAssembly(P, sequences) -> cset (Section 4.4): walks every chain and
 * concatenates l_r[alpha:pre(e0)] + l_c1[post(e0):pre(e1)] + ... +
 * l_r'[post(e_{q-2}):beta]: each read but the last contributes its part before
 * the overlap with the next read (in its walking orientation), the last read
 * contributes all of its bases.  A path starts at its smaller-id root; a cycle
 * starts at its smallest read, steps to that read's smaller-id neighbour and
 * does not traverse its closing edge.  The first read's orientation is the s
 * bit of the first edge, every other read's the d bit of the edge it is
 * entered by.  Fills `out` (cg_contigs above). */
int cg_assemble(cg_ctx *ctx, const cg_graph *g, const cg_parts *parts, const cg_local *local,
                int32_t P, const cg_contigs *out, void *stream);

/* ---- without allocation ---------------------------------------------------- */

/* Capacity of the allocation-free entry point: the graph's context scratch
 * (cg_footprint's `scratch` figure) must fit in this many bytes. */
#define CG_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* ContigGeneration on one graph without a context and without allocating:
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Runs
 * cg_mask_branches, cg_components, cg_partition, cg_induce and cg_assemble in
 * that order on `stream` with the same kernels, and fills the same outputs
 * (arguments as in those calls).  The scratch the steps need lives in a static
 * device array of the library, CG_NOALLOC_SCRATCH_BYTES plus a few KB, one
 * copy per GPU, held until the process ends; the call makes no allocation
 * of any kind.  The first call on a device looks up that device's copy.
 * d_status [device, optional] receives the CG_STATUS_* bits the call raised.
 * Errors (before anything is enqueued): as the five calls; CG_EUNSUPPORTED
 * when the graph needs more scratch than CG_NOALLOC_SCRATCH_BYTES.
 * All calls on one GPU share its array, which keeps the last call's contents
 * (each call clears what must start at zero): calls that overlap in time on
 * one GPU (other streams or threads) race and give undefined results; calls
 * one after another on one stream are safe. */
int cg_contig_generation_noalloc(const cg_graph *g, int32_t P, int32_t min_reads, int32_t weight,
                                 uint8_t *flags, int32_t *d_counts, int32_t *label,
                                 const cg_parts *parts, const cg_local *local,
                                 const cg_contigs *contigs, uint32_t *d_status, void *stream);

/* ---- batched form -------------------------------------------------------- */

/* One graph of a batch: its inputs, its parameters and the same output
 * buffers the single-graph calls fill (same sizes and meaning).  The batched
 * kernels move reads with 16-byte accesses: g.row_ptr, flags, label and
 * parts.label_comp must be 16-byte aligned. */
typedef struct {
  cg_graph g;
  int32_t P;          /* bins, 1..65536 */
  int32_t min_reads;  /* as in cg_partition */
  int32_t weight;     /* as in cg_partition: CG_WEIGHT_READS or CG_WEIGHT_BASES */
  uint8_t *flags;     /* [n]  as in cg_mask_branches */
  int32_t *d_counts;  /* [2]  as in cg_mask_branches */
  int32_t *label;     /* [n]  as in cg_components */
  cg_parts parts;
  cg_local local;
  cg_contigs contigs;
} cg_job;

/* Launch shapes of the batched kernels (0 = default).  They change speed,
 * never results. */
/* Every output buffer of one job carved from one device buffer: with base
 * NULL, *bytes [host] receives the bytes needed; with base [device, 256-byte
 * aligned, at least that many bytes] the output pointers of *job [host]
 * (flags, d_counts, label, parts, local, contigs with cap_words) are set to
 * buffers inside it, each at a 256-byte boundary, at the capacities the
 * five calls state for a graph of n reads and P bins (as cg_footprint's
 * outputs, plus the alignment).  The graph, P, min_reads and weight of *job
 * are left alone.  Errors: CG_EINVAL. */
int cg_job_outputs(int32_t n, int32_t P, uint64_t cap_words, void *base, uint64_t *bytes,
                   cg_job *job);

typedef struct {
  int32_t vertex_tile;     /* vertices per workgroup in vertex passes: 256 (default), 512, 1024 */
  int32_t copy_block;      /* threads per workgroup of the base copy, multiple of 64 (256);
                              the copy runs one wave per chunk of 32 pieces */
  int32_t persist_blocks;  /* workgroups of the persistent per-component passes (4 per
                              compute unit; the one-wave passes take 4x as many), each
                              capped at the workgroups that fit on the device at once */
} cg_batch_params;

typedef struct cg_batch cg_batch;

/* Plan a batch of n_jobs independent graphs (jobs is [host]): copies the job
 * descriptors to the device and allocates the tile table, scan state and
 * per-job scratch (device memory owned by the batch).  The buffers the jobs
 * point to must stay valid and unmoved while the batch exists.  Runs every
 * step of Algorithm 2 for all jobs with one launch per phase; each job's
 * outputs are identical to the five single-graph calls on that job.  A job
 * with more than 32768 directed entries is run by the single-graph kernels,
 * in the same launch sequence ahead of the batched launches. */
int cg_batch_create(cg_ctx *ctx, int32_t n_jobs, const cg_job *jobs,
                    const cg_batch_params *params, cg_batch **out);

/* Device bytes a batch of these jobs needs (as cg_batch_create allocates;
 * vertex_tile of params counts, NULL params means the defaults).  Only each
 * job's g.n, g.m, P and weight are read: its pointers may be NULL, so a
 * caller can size a batch before it allocates the jobs' outputs.  bytes is
 * [host]. */
int cg_batch_bytes(int32_t n_jobs, const cg_job *jobs, const cg_batch_params *params,
                   uint64_t *bytes);

/* A batch with `bytes` of device memory and no jobs yet, for a caller that
 * plans batch after batch into the same memory (a serving loop): give it
 * jobs with cg_batch_plan. */
int cg_batch_create_empty(cg_ctx *ctx, uint64_t bytes, const cg_batch_params *params,
                          cg_batch **out);

/* Replace the batch's jobs (same checks as cg_batch_create), within its
 * memory: CG_ECAPACITY when they need more than it has (cg_batch_bytes), and
 * nothing changes.  The job tables are uploaded on `stream`; the batch's
 * earlier work must be complete (the new jobs reuse its memory).  A captured
 * graph of the batch is dropped. */
int cg_batch_plan(cg_batch *b, int32_t n_jobs, const cg_job *jobs, void *stream);

/* Enqueue the whole path for every job of the batch on `stream`. */
int cg_batch_run(cg_batch *b, void *stream);

/* Results of the batch, for a caller that downloads them (enqueue after
 * cg_batch_run or cg_batch_launch, on the same stream).
 *
 * cg_batch_counts writes d_counts [device, 4 n_jobs + 1 int64]: for job j
 * (plan order) 4j: contigs nc (*d_n_comp), 4j+1: layout entries ne
 * (d_sizes[0]), 4j+2: base words tw (*d_total_words, at most cap_words),
 * 4j+3: the byte offset of the job's packed results; 4 n_jobs: their total
 * bytes.
 *
 * cg_batch_pack copies every job's results, trimmed to those counts, into
 * d_dst [device, 16-byte aligned] at the job's offset, as one packed record:
 *   len u64[nc], base_off u64[nc], label, bin, start, n_reads, cflags,
 *   layout_off (4 bytes each)[nc], layout_vid i32[ne], bases u32[tw],
 *   layout_rev u8[ne], zero bytes up to a multiple of 16.
 * Nothing is written past dst_bytes: a caller that read the total first
 * (d_counts[4 n_jobs]) passes at least that.  Errors: CG_EINVAL. */
int cg_batch_counts(cg_batch *b, int64_t *d_counts, void *stream);
int cg_batch_pack(cg_batch *b, const int64_t *d_counts, void *d_dst, uint64_t dst_bytes,
                  void *stream);

/* Capture cg_batch_run into a HIP graph on `stream` (must not be the NULL
 * stream) and instantiate it; cg_batch_launch then replays it. */
int cg_batch_capture(cg_batch *b, void *stream);
int cg_batch_launch(cg_batch *b, void *stream);

/* Release the batch (the caller makes sure none of its work is in flight). */
int cg_batch_destroy(cg_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* CG_H */
