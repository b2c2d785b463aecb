// Internal declarations of libcg: context layout, scratch carving, device
// utilities (wave / block scans, the single-pass look-back scan) and the
// kernel launchers each step's source file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include "../../include/cg.h"

namespace cg {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Fixed device state of a context: small counters that kernels clean up
// themselves after use, so that every launch finds them zero.
// ---------------------------------------------------------------------------
// Workgroups of the plain mask pass at most (it strides over the reads).
constexpr int kMaskMaxBlocks = 1024;

struct Fixed {
  // per workgroup of the mask pass: branch reads (low 32 bits), kept entries
  // (high 32)
  unsigned long long mask_part[kMaskMaxBlocks];
  unsigned int mask_ticket;  // workgroups done, for grids that sum in the kernel
  unsigned int status;             // CG_STATUS_* bits
  unsigned long long valid_best;   // packed first failure of cg_validate
  unsigned int scan_ticket;        // look-back scan: block ticket
  unsigned int scan_done;          // look-back scan: exited blocks
  unsigned int pad[8];
};

// Items per block of the look-back scan (one item per thread).
constexpr int kScanBlock = 1024;

struct Scratch {
  unsigned long long *scan_status;  // [scan_blocks]
  int32_t *tmp;        // [2n] induce: reads bucketed by component (the batched form:
                       // (id, tile-list slot) pairs)
  int32_t *lidx;       // [n] induce: local number of each read
  uint32_t *fill;      // [n] induce: bucket cursors
  uint64_t *piece_off; // [n] assemble: base offset of each piece in its contig
  uint32_t *piece_len; // [n] assemble: bases of each piece
  uint64_t *piece_src; // [n] assemble: where each piece starts in the store (see piece_anchor)
  int32_t *lay_contig; // [n] assemble: record index of each layout entry
  uint64_t *keys;      // [2n] partition fallback: sort keys
  uint64_t *bins;      // [2P] partition fallback: sorted bin keys
  int32_t *aux;        // [n] partition fallback: bin of each component
  int32_t *walk;       // [16n] assemble: chain arrays of components too big for LDS
  int32_t *estart;     // [n] batched induce: first local CSR entry of each component
  int32_t *memb;       // [n] batched components: first member slot of each component
  uint64_t *comp_w;    // [n] partition: bases weight of each component
  uint64_t *bin_reads; // [P] partition: reads of each bin
};

}  // namespace cg

namespace cg {
struct ProfEntry {
  const char *name;
  hipEvent_t a, b;
};
}  // namespace cg

struct cg_ctx {
  int device;
  char *scratch;
  size_t scratch_bytes;
  cg::Fixed *fixed;
  // optional per-kernel event timing (cg_ctx_profile)
  int prof_cap;
  int prof_used;
  long long prof_dropped;
  cg::ProfEntry *prof;
};

namespace cg {

// Scratch carving shared by cg_footprint, the calls and the batch slices.
struct Layout {
  size_t scan_status, tmp, lidx, fill, piece_off, piece_len, lay_contig, keys, bins, aux, walk,
      estart, memb, piece_src, comp_w, bin_reads, total;
};
Layout layout(int64_t n, int64_t m, int64_t P);
bool carve(cg_ctx *ctx, int64_t n, int64_t m, int64_t P, Scratch *s);

// error text (thread local) and HIP error translation
int set_error(int code, const char *fmt, ...);
int hip_check(hipError_t e, const char *what);

// host-side argument checks shared by the entry points
int check_graph(const cg_graph *g, bool need_seq);
int check_P(int32_t P);
int check_parts(const cg_parts *p);
int check_local(const cg_local *l);
int check_contigs(const cg_contigs *c);

// ---------------------------------------------------------------------------
// Device utilities
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Device global memory.  Pointers a kernel reads out of a descriptor in
// memory are generic to the compiler; typing them as global lets it use
// global (not flat) memory instructions.
#define CG_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ int ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int32_t *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = __shfl_up(x, d);
    if (l >= d) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
  return x;
}

// A workgroup barrier that orders LDS accesses only: global loads and
// stores stay in flight across it (a full barrier also waits for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block-wide exclusive scan; returns the exclusive prefix, *total the block
// sum.  `sh` needs BLOCK/64 + 1 entries of T.  All threads must call it.
// kLdsOnly: its barriers order LDS only (the caller's global accesses stay
// in flight); a one-wave block needs neither LDS nor barriers.
template <typename T, int BLOCK, bool kLdsOnly = false>
__device__ __forceinline__ T block_excl_scan(T x, T *sh, T *total) {
  constexpr int NW = BLOCK / kWave;
  const int w = threadIdx.x / kWave, l = lane_id();
  T inc = wave_incl_scan(x);
  if constexpr (kLdsOnly && BLOCK == kWave) {
    *total = __shfl(inc, kWave - 1);
    (void)sh;
    (void)w;
    (void)l;
    return inc - x;
  }
  auto bar = [] {
    if constexpr (kLdsOnly) lds_barrier();
    else __syncthreads();
  };
  if (l == kWave - 1) sh[w] = inc;
  bar();
  if (w == 0) {
    T v = l < NW ? sh[l] : T(0);
    T vi = wave_incl_scan(v);
    if (l < NW) sh[l] = vi - v;
    if (l == NW - 1) sh[NW] = vi;
  }
  bar();
  T r = sh[w] + inc - x;
  *total = sh[NW];
  bar();
  return r;
}

// Single-pass decoupled look-back scan over `n_items` items, one per thread,
// blocks of kScanBlock.  Block order comes from an atomic ticket, so a block
// only waits on blocks that already run.  The last block to exit resets the
// ticket, the exit counter and the status words, so the next launch finds
// them zero.  status words: bits 63..62 = 0 none / 1 block aggregate /
// 2 inclusive prefix, bits 61..0 = value.
struct ScanCtx {
  unsigned long long *status;
  unsigned int *ticket;
  unsigned int *done;
  unsigned int *error;  // CG_STATUS_* word raised if a look-back gives up
};

// Polls of a predecessor's status before a look-back gives up (raising
// CG_STATUS_SCAN_STALLED); far beyond any real wait, it only bounds a wait
// that would otherwise never end.
constexpr long long kLookbackSpinLimit = 1ll << 26;

constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagPre = 2ull << 62;
constexpr unsigned long long kValMask = (1ull << 62) - 1;

// Block ticket of a look-back scan launch (all threads of the block call it).
__device__ __forceinline__ int lookback_ticket(ScanCtx sc) {
  __shared__ int blk;
  if (threadIdx.x == 0) blk = (int)atomicAdd(sc.ticket, 1u);
  __syncthreads();
  return blk;
}

__device__ __forceinline__ unsigned long long atomic_ld64(unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish the block aggregate, look back, publish the inclusive prefix;
// returns the exclusive prefix of the block.  Called by every lane of the
// block's first wave (the result is the same in every lane).
//
// The look-back reads a window of 64 predecessors at once, one per lane:
// the nearest one holding an inclusive prefix ends the walk, and the
// aggregates of the lanes before it are added to it; a window of aggregates
// only adds all 64 and moves 64 blocks back.  (One predecessor per step made
// block k wait about k round trips when all blocks start together.)  A status
// word carries its flag and value in one 64-bit atomic and nothing else is
// read through it, so relaxed device-scope atomics suffice: no L2 write-back
// per publish and no L2 invalidation per poll.
__device__ __forceinline__ unsigned long long lookback_publish(ScanCtx sc, int blk,
                                                               unsigned long long agg,
                                                               int seg_first = 0) {
  const int lane = lane_id();
  if (blk == seg_first) {
    if (lane == 0)
      __hip_atomic_store(&sc.status[blk], kFlagPre | agg, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0)
    __hip_atomic_store(&sc.status[blk], kFlagAgg | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned long long excl = 0;
  int top = blk - 1;
  long long spins = 0;
  while (true) {
    // the segment's first block publishes an inclusive prefix, so no window
    // needs a block before it
    const int p = top - lane;
    const unsigned long long s = p >= seg_first ? atomic_ld64(&sc.status[p]) : kFlagPre;
    const unsigned long long f = s & ~kValMask;
    const uint64_t pre = __ballot(f == kFlagPre);
    const uint64_t none = __ballot(f == 0);
    // lanes up to and including the nearest inclusive prefix (all if none)
    const uint64_t upto = pre ? (pre ^ (pre - 1)) : ~0ull;
    if (none & upto) {  // a predecessor has not published yet (it is running)
      if (++spins < kLookbackSpinLimit) continue;
      if (lane == 0) atomicOr(sc.error, CG_STATUS_SCAN_STALLED);
      break;
    }
    unsigned long long v = ((upto >> lane) & 1ull) ? (s & kValMask) : 0ull;
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    excl += v;
    if (pre) break;
    top -= kWave;
  }
  if (lane == 0)
    __hip_atomic_store(&sc.status[blk], kFlagPre | (excl + agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// Called by every thread of every block at the very end of a look-back scan
// kernel: the last block out clears the state for the next launch.  The exit
// count is a release, so a block's status stores are done before the last
// block can clear them.
__device__ __forceinline__ void lookback_finish(ScanCtx sc, int nblocks) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned d = __hip_atomic_fetch_add(sc.done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    last = (d == (unsigned)nblocks - 1);
    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (last) {
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) sc.status[i] = 0;
    if (threadIdx.x == 0) {
      *sc.ticket = 0;
      *sc.done = 0;
    }
    __threadfence();
  }
}

// Block-wide exclusive scan of one item per thread with the look-back
// across blocks.  `val` is this thread's item value.  Returns the exclusive
// prefix; *total receives the sum over all blocks up to and including this
// one (the grand total in the last block).
template <int BLOCK = kScanBlock>
__device__ __forceinline__ unsigned long long lookback_block_scan(ScanCtx sc, int blk,
                                                                  unsigned long long val,
                                                                  unsigned long long *incl_end,
                                                                  int seg_first = 0) {
  __shared__ unsigned long long sh[BLOCK / kWave + 1];
  __shared__ unsigned long long base;
  unsigned long long agg;
  unsigned long long ex = block_excl_scan<unsigned long long, BLOCK>(val, sh, &agg);
  if (threadIdx.x < kWave) {
    const unsigned long long b = lookback_publish(sc, blk, agg, seg_first);
    if (threadIdx.x == 0) base = b;
  }
  __syncthreads();
  *incl_end = base + agg;
  return base + ex;
}

// Kernel launch, bracketed by two events on its stream when the context's
// per-kernel timing is on.
int prof_begin(cg_ctx *ctx, hipStream_t st, const char *name);
void prof_end(cg_ctx *ctx, hipStream_t st, int slot);

// A roctx range over a scope: the host-side enqueue of one step of
// Algorithm 2 (a tracer such as rocprofv3 --marker-trace shows it beside the
// step's kernels).  Costs a call when no tracer is attached.
struct PhaseRange {
  explicit PhaseRange(const char *name) { roctxRangePushA(name); }
  ~PhaseRange() { roctxRangePop(); }
  PhaseRange(const PhaseRange &) = delete;
  PhaseRange &operator=(const PhaseRange &) = delete;
};

#define CG_LAUNCH(ctx, kern, grid, block, st, ...)                 \
  do {                                                             \
    const int cg_prof_slot_ = ::cg::prof_begin((ctx), (st), #kern); \
    hipLaunchKernelGGL(kern, grid, block, 0, st, __VA_ARGS__);     \
    ::cg::prof_end((ctx), (st), cg_prof_slot_);                    \
  } while (0)

// ---------------------------------------------------------------------------
// Launchers (one per step; each returns CG_OK or an error code)
// ---------------------------------------------------------------------------
int launch_validate(cg_ctx *ctx, const cg_graph &g, int64_t *d_bad, hipStream_t st);
int launch_mask(cg_ctx *ctx, const cg_graph &g, uint8_t *flags, int32_t *d_counts,
                hipStream_t st);
int launch_components(cg_ctx *ctx, const cg_graph &g, const uint8_t *flags, int32_t *label,
                      hipStream_t st);
int launch_partition(cg_ctx *ctx, const cg_graph &g, const Scratch &s, const uint8_t *flags,
                     const int32_t *label, int32_t P, int32_t min_reads, int32_t weight,
                     const cg_parts &out, hipStream_t st);
int launch_induce(cg_ctx *ctx, const cg_graph &g, const Scratch &s, const uint8_t *flags,
                  const int32_t *label, const cg_parts &parts, int32_t P, const cg_local &out,
                  hipStream_t st);
int launch_assemble(cg_ctx *ctx, const cg_graph &g, const Scratch &s, const cg_parts &parts,
                    const cg_local &local, int32_t P, const cg_contigs &out, hipStream_t st);
int launch_reduce(cg_ctx *ctx, const cg_graph &g, const Scratch &s, uint32_t fuzz,
                  uint8_t *contained, uint8_t *kept, int32_t *s_row_ptr, int32_t *s_col,
                  uint32_t *s_ovl, uint8_t *s_strand, int32_t *d_m, hipStream_t st);

inline ScanCtx scan_ctx(cg_ctx *ctx, const Scratch &s) {
  return ScanCtx{s.scan_status, &ctx->fixed->scan_ticket, &ctx->fixed->scan_done,
                 &ctx->fixed->status};
}

inline int scan_blocks(int64_t items) { return (int)((items + kScanBlock - 1) / kScanBlock); }

}  // namespace cg
