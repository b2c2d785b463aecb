// Batched form: the five steps of Algorithm 2 for many independent string
// graphs ("jobs") with one launch per phase for the whole batch.
//
//  mask + comps    one workgroup per job, largest first: branch flags,
//                  components and the component table from LDS bitmaps
//  vertex passes   each job is cut into tiles of T vertices; a launch covers
//                  the tiles of every job (tile -> job table)
//  component and   persistent grids over the batch-wide item ranges
//  piece passes    (components, pieces) whose per-job bases the last LPT
//                  workgroup computes on the device; the per-component passes
//                  take a work queue of every component of the batch in
//                  decreasing read count
//
// Every counter a launch uses is reset by the launch itself, so the
// launches (ten, or eleven when a job partitions by bases weights) can be
// captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "cg_device.h"

namespace cg {

struct BJob {
  cg_graph g;
  int32_t P, min_reads, weight;
  uint8_t *flags;
  int32_t *counts;
  int32_t *label;
  cg_parts parts;
  cg_local local;
  cg_contigs out;
  Scratch s;
  int32_t vt_first, vt_count;  // the job's vertex tiles (covering 0..n)
  int32_t mt_first, mt_count;  // the job's mask tiles (kb_mask_tiles)
  int32_t external;            // 1: the job runs through the single-graph kernels before the
                               // batched launches, which then leave it alone
  int32_t pad_;
};

// A job's descriptor by value.  The job table is read-only while a launch
// runs, so it is read through the constant address space: with a uniform job
// index the fields arrive by scalar loads, and no LDS store can alias them.
#define CG_CONST __attribute__((address_space(4)))
static_assert(sizeof(BJob) % 8 == 0, "job descriptors are copied in 8-byte words");
__device__ __forceinline__ BJob job_at(const BJob *jobs, int j) {
  BJob out;
  const CG_CONST uint64_t *p = (const CG_CONST uint64_t *)(jobs + j);
  uint64_t *q = reinterpret_cast<uint64_t *>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(BJob) / 8); ++k) q[k] = p[k];
  return out;
}
// the same for the batch-wide tables that an earlier launch wrote
__device__ __forceinline__ int32_t ld_const(const int32_t *a, int64_t i) {
  return ((const CG_CONST int32_t *)a)[i];
}

// A work-queue entry: a component, its job, and what its per-component
// passes need of the component table, so that none of it is a load of its
// own on the component's critical path.
struct WqE {
  int32_t job, c, q, st;  // job, component, reads, first local number
  int32_t estart;         // its first local CSR entry
  int32_t rank;           // its contig record (the component's (bin, label) rank)
  const int32_t *mem;     // its member records (id, list slot | kept bits << 30)
};
static_assert(sizeof(WqE) == 32, "queue entries are read as 32 bytes");

struct BatchDev {
  BJob *jobs;                       // [n_jobs]
  int32_t *tile_job;                // [n_vtiles]
  int32_t *comp_base;               // [n_jobs + 1] first component item of each job
  int32_t *piece_base;              // [n_jobs + 1] first piece item of each job
  int32_t *chunk_base;              // [n_jobs + 1] first copy chunk of each job
  int32_t *chunk_cp;                // [n_jobs] pieces per copy chunk of each job
  int2 *job_cnt;                    // [n_jobs] (components, component reads) of each job
  // work queue of the per-component passes: every component of the batch,
  // in decreasing read count
  WqE *wq;                          // [upper bound on the batch's components]
  int32_t *wq_hist;                 // [kWqBuckets] components per read count (capped)
  int32_t *wq_cur;                  // [kWqBuckets] placement cursors
  int32_t *wq_meta;                 // [8] 0: components, 1: those above kWalkSmallCap
                                    // reads, 2: above kIwCap, 3: above kWalkTinyCap
  int32_t *comp_job;                // [sum n] job of each batch-wide component
  int4 *chunk_desc;                 // [bound on the chunks] copy chunk: job, first piece,
                                    // pieces (0: the job's bases overflowed), job's pieces
  unsigned int *counters;           // [8] 2: LPT ticket
  const int32_t *job_order;         // [n_jobs] jobs by decreasing read count
  int2 *mt_cnt;                     // [n_mtiles] (listed reads, branch reads) of each mask tile
  Fixed *fixed;
  int32_t n_jobs, n_vtiles, n_mtiles;
};

// index j with base[j] <= i < base[j+1] (base ascending, base[0] = 0; of
// several jobs with the same base, the last, which is the one holding i)
__device__ __forceinline__ int job_of(const int32_t *__restrict__ base, int n_jobs, int32_t i) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// 1a. The reads of every job in tiles of kMaskTile, over the whole chip
// (one workgroup's share of a job would get a sliver of the memory
// bandwidth while all jobs stream at once): degree from row_ptr, the
// "listed" (degree 1 or 2, the only reads that can keep an entry) and
// "branch" (degree >= 3) bitmaps of the job, and every listed read with its
// columns, packed per tile in id order by a block scan.  It also stores every
// read's flags, label and label_comp as they are for a read the components
// step leaves alone (the branch bit, its own id, -1), so that step, one
// workgroup per job, stores only what its listed reads change.
// ---------------------------------------------------------------------------
struct MaskTile {
  const int32_t *row_ptr;
  const int32_t *col;
  int4 *list;        // the job's listed reads: tile t's at list[t * kMaskTile], as
                     // (id, first column, second column or -1, first entry)
  uint32_t *bits;    // the job's bitmaps: W listed words, then W branch words
  int2 *tile_cnt;    // (listed reads, branch reads) of this tile
  uint8_t *flags;    // the job's outputs, given their defaults here (below)
  int32_t *label;
  int32_t *label_comp;
  int32_t n, v0, W, pad_;
};
static_assert(sizeof(MaskTile) % 8 == 0, "tile descriptors are copied in 8-byte words");

constexpr int kMaskThreads = 256;
constexpr int kMaskGroups = 2;  // groups of 4 consecutive reads per thread
constexpr int kMaskTile = 4 * kMaskThreads * kMaskGroups;
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kMaskThreads) void kb_mask_tiles(const MaskTile *__restrict__ tiles) {
  __shared__ int64_t sh[kMaskThreads / kWave + 1];
  MaskTile D;
  {
    const CG_CONST uint64_t *p = (const CG_CONST uint64_t *)(tiles + blockIdx.x);
    uint64_t *q = reinterpret_cast<uint64_t *>(&D);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(MaskTile) / 8); ++k) q[k] = p[k];
  }
  const CG_GLOBAL int32_t *rp = (const CG_GLOBAL int32_t *)D.row_ptr;
  const CG_GLOBAL int32_t *col = (const CG_GLOBAL int32_t *)D.col;
  CG_GLOBAL i32x4 *list = (CG_GLOBAL i32x4 *)D.list;
  CG_GLOBAL uint32_t *bits = (CG_GLOBAL uint32_t *)D.bits;
  const int32_t n = D.n;
  const int lane = lane_id();
  // every load issued before any is used: a group past the end loads the
  // last whole group instead and is patched or ignored below
  const int32_t last4 = n >= 3 ? (n - 3) & ~3 : 0;
  int32_t v0[kMaskGroups];
  i32x4 a[kMaskGroups];
  int32_t e4[kMaskGroups];
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g) {
    v0[g] = D.v0 + g * 4 * kMaskThreads + 4 * (int32_t)threadIdx.x;
    a[g] = i32x4{0, 0, 0, 0};
    if (n >= 3) a[g] = *(const CG_GLOBAL i32x4 *)(rp + (v0[g] + 3 <= n ? v0[g] : last4));
    e4[g] = rp[lane == kWave - 1 && v0[g] + 4 <= n ? v0[g] + 4 : 0];
  }
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g) {
    if (v0[g] + 3 > n && v0[g] <= n) {  // the job's last, partial group
      a[g].x = rp[v0[g]];
      if (v0[g] + 1 <= n) a[g].y = rp[v0[g] + 1];
      if (v0[g] + 2 <= n) a[g].z = rp[v0[g] + 2];
    }
  }
  constexpr int R = 4 * kMaskGroups;
  int32_t dg[R], rs[R];
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g) {
    const int32_t nx = __shfl_down(a[g].x, 1);
    const int32_t r[5] = {a[g].x, a[g].y, a[g].z, a[g].w, lane == kWave - 1 ? e4[g] : nx};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dg[4 * g + i] = v0[g] + i < n ? r[i + 1] - r[i] : 0;
      rs[4 * g + i] = r[i];
    }
  }
  // columns of the listed reads (rows of consecutive reads are consecutive)
  int32_t u0[R], u1[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    u0[k] = (dg[k] == 1 || dg[k] == 2) ? col[rs[k]] : -1;
    u1[k] = dg[k] == 2 ? col[rs[k] + 1] : -1;
  }
  // the bitmaps: a group's 4 reads are a nibble of word v0 / 32; eight lanes
  // OR their nibbles into a word
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g) {
    uint32_t ln = 0, bn = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ln |= (dg[4 * g + i] == 1 || dg[4 * g + i] == 2 ? 1u : 0u) << i;
      bn |= (dg[4 * g + i] >= 3 ? 1u : 0u) << i;
    }
    uint32_t lb = ln << (4 * (lane & 7)), bb = bn << (4 * (lane & 7));
    lb |= __shfl_xor(lb, 1);
    bb |= __shfl_xor(bb, 1);
    lb |= __shfl_xor(lb, 2);
    bb |= __shfl_xor(bb, 2);
    lb |= __shfl_xor(lb, 4);
    bb |= __shfl_xor(bb, 4);
    const int32_t w = v0[g] >> 5;
    if ((lane & 7) == 0 && w < D.W) {
      bits[w] = lb;
      bits[D.W + w] = bb;
    }
  }
  // the defaults of every read (16-byte stores of whole groups)
  {
    CG_GLOBAL uint8_t *fl = (CG_GLOBAL uint8_t *)D.flags;
    CG_GLOBAL int32_t *lab = (CG_GLOBAL int32_t *)D.label;
    CG_GLOBAL int32_t *lc = (CG_GLOBAL int32_t *)D.label_comp;
#pragma unroll
    for (int g = 0; g < kMaskGroups; ++g) {
      const int32_t v = v0[g];
      uint32_t f = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) f |= (dg[4 * g + i] >= 3 ? 1u : 0u) << (8 * i);
      if (v + 3 < n) {
        *(CG_GLOBAL uint32_t *)(fl + v) = f;
        *(CG_GLOBAL i32x4 *)(lab + v) = i32x4{v, v + 1, v + 2, v + 3};
        *(CG_GLOBAL i32x4 *)(lc + v) = i32x4{-1, -1, -1, -1};
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (v + i < n) {
            fl[v + i] = (uint8_t)(f >> (8 * i));
            lab[v + i] = v + i;
            lc[v + i] = -1;
          }
      }
    }
  }
  // listed reads packed in id order: group 0 of every thread precedes group
  // 1, so one scan of (listed, branch) counts of both groups, 16-bit fields
  // (a tile holds fewer than 2^16 reads), gives every position
  static_assert(kMaskGroups == 2, "two groups per scan");
  int64_t cnt = 0;
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g) {
    int64_t c = 0, b = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      c += (dg[4 * g + i] == 1 || dg[4 * g + i] == 2) ? 1 : 0;
      b += dg[4 * g + i] >= 3 ? 1 : 0;
    }
    cnt |= (c | (b << 16)) << (32 * g);
  }
  int64_t tot;
  const int64_t ex = block_excl_scan<int64_t, kMaskThreads>(cnt, sh, &tot);
  const int32_t listed0 = (int32_t)(tot & 0xFFFF);
  int32_t pos[kMaskGroups] = {D.v0 + (int32_t)(ex & 0xFFFF),
                              D.v0 + listed0 + (int32_t)((ex >> 32) & 0xFFFF)};
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * g + i;
      if (dg[k] == 1 || dg[k] == 2) list[pos[g]++] = i32x4{v0[g] + i, u0[k], u1[k], rs[k]};
    }
  if (threadIdx.x == 0) {
    CG_GLOBAL int32_t *tc = (CG_GLOBAL int32_t *)D.tile_cnt;
    tc[0] = listed0 + (int32_t)((tot >> 32) & 0xFFFF);
    tc[1] = (int32_t)((tot >> 16) & 0xFFFF) + (int32_t)((tot >> 48) & 0xFFFF);
  }
}

// ---------------------------------------------------------------------------
// 1. BranchRemoval, ConnectedComponent and the component table of each job in
// one workgroup (Sections 4.2 and 4.3), largest jobs dispatched first.
//
// A job's reads are cut into words of 32 consecutive reads and each thread
// owns a contiguous run of words, so its reads, and the local numbers of its
// listed reads (below), are contiguous and in id order.  A thread's work
// follows what its words hold: a word without a read of degree 1-2 costs a
// few instructions for all 32 reads.
//  A  row_ptr of the thread's words: the bitmaps "listed" (degree 1 or 2,
//     the only reads that can keep an entry) and "branch" (degree >= 3)
//  B  listed reads before each word (one block scan): a listed read's local
//     number is its rank among the job's listed reads, so local numbers
//     follow read ids
//  C  each listed read's entries: kept when the other end is not a branch
//     read; the other end's local number from the bitmaps
//  D  union-find over local numbers (larger root under smaller, so a root is
//     its component's smallest id): a read first points at its smallest kept
//     neighbour below it, and only an edge that leaves open is hooked
//  E  roots and per-root counts (4 per read + 1 per path end)
//  H  flags, labels and label_comp: what a read of degree 1-2 changes of the
//     defaults the tile pass stored (when one-read components are eligible,
//     every read's, with their numbering)
//  F  eligible components in label order (one scan over the threads' runs)
//     and each component's members grouped for the induce step
// The listed reads' state (entry, forest/counter, hook/root) is in LDS, or
// in the job's scratch for a job with more listed reads than LDS holds.
// ---------------------------------------------------------------------------
constexpr int kMcBlock = 1024;
constexpr int kMcReadCap = 131072;               // reads of a job (LDS bitmaps)
constexpr int kMcWords = kMcReadCap / 32;
constexpr int kMcMaxWpt = kMcWords / kMcBlock;   // words per thread at most
constexpr int kMcListCap = 9216;                 // listed reads held in LDS
constexpr int kMcPer = kMcListCap / kMcBlock;    // listed reads per thread at most in LDS
// jobs with more directed entries or reads go through the single-graph
// kernels (with at most this many entries a job's listed reads fit in LDS
// unless most of its reads have degree 1)
constexpr int64_t kExternalEntries = 2 * (int64_t)kMcListCap;
constexpr int32_t kNotEligible = -(1 << 30);
constexpr uint32_t kIdMask = (1u << 30) - 1;     // low bits of a listed read's entry: its id

__device__ __forceinline__ uint8_t kind_of(uint32_t c4) {
  return (c4 >> 2) == 1 ? CG_KIND_SINGLE : ((c4 & 3u) ? CG_KIND_PATH : CG_KIND_CYCLE);
}

// Listed reads' state: entry (id | kept bits << 30); `a`: forest parent, then
// per-root counter, then member cursor; `b`: hook target, then root (or
// ~component for a numbered root).  In LDS, or in the job's scratch.
template <bool kLds>
struct McArr;
template <>
struct McArr<true> {
  uint32_t *lid;
  int32_t *a;
  int32_t *b;
  static constexpr bool lds = true;
};
template <>
struct McArr<false> {
  CG_GLOBAL uint32_t *lid;
  CG_GLOBAL int32_t *a;
  CG_GLOBAL int32_t *b;
  static constexpr bool lds = false;
};

// relaxed atomics of the union-find: workgroup scope in LDS; device scope in
// global memory
__device__ __forceinline__ int32_t mc_ld(int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int32_t mc_ld(CG_GLOBAL int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void mc_st(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void mc_st(CG_GLOBAL int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool mc_cas(int32_t *p, int32_t *expect, int32_t v) {
  return __hip_atomic_compare_exchange_strong(p, expect, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ bool mc_cas(CG_GLOBAL int32_t *p, int32_t *expect, int32_t v) {
  return __hip_atomic_compare_exchange_strong(p, expect, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t mc_add(int32_t *p, int32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int32_t mc_add(CG_GLOBAL int32_t *p, int32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename P>
__device__ __forceinline__ int32_t mc_find(P par, int32_t x) {
  while (true) {
    const int32_t p = mc_ld(par + x);
    if (p == x) return x;
    const int32_t gp = mc_ld(par + p);
    if (gp == p) return p;
    mc_st(par + x, gp);  // path halving: gp is an ancestor of x
    x = gp;
  }
}

// link the larger root under the smaller one; a failed link climbs to the
// parent the root got meanwhile
template <typename P>
__device__ __forceinline__ void mc_union(P par, int32_t a, int32_t b) {
  a = mc_find(par, a);
  b = mc_find(par, b);
  while (a != b) {
    const int32_t hi = a > b ? a : b, lo = a > b ? b : a;
    int32_t expect = hi;
    if (mc_cas(par + hi, &expect, lo)) return;
    if (a == hi) a = expect;
    else b = expect;
  }
}

// The job's outputs and scratch arrays this kernel writes, typed as global
// memory: stores through generic pointers would be flat stores, which the
// LDS wait counter also counts, so every later LDS wait would wait for them.
struct McOut {
  CG_GLOBAL uint8_t *flags;
  CG_GLOBAL int32_t *label;
  CG_GLOBAL int32_t *label_comp;
  CG_GLOBAL int32_t *comp_label;
  CG_GLOBAL int32_t *comp_size;
  CG_GLOBAL uint8_t *comp_kind;
  CG_GLOBAL int32_t *memb;
  CG_GLOBAL uint64_t *comp_w;
  CG_GLOBAL int32_t *tmp;
};

__device__ __forceinline__ McOut mc_out(const BJob &J) {
  return McOut{(CG_GLOBAL uint8_t *)J.flags,          (CG_GLOBAL int32_t *)J.label,
               (CG_GLOBAL int32_t *)J.parts.label_comp, (CG_GLOBAL int32_t *)J.parts.comp_label,
               (CG_GLOBAL int32_t *)J.parts.comp_size, (CG_GLOBAL uint8_t *)J.parts.comp_kind,
               (CG_GLOBAL int32_t *)J.s.memb,          (CG_GLOBAL uint64_t *)J.s.comp_w,
               (CG_GLOBAL int32_t *)J.s.tmp};
}

// Member slot `at` of a component: the read's id and where the tile list
// holds it (its slot | kept bits << 30), or kNoSlot where the list does not
// (a read without kept entries, or a job whose listed reads' state is in
// scratch, which reuses the list's memory).  One 8-byte store.
constexpr int32_t kNoSlot = (1 << 30) - 1;
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void mc_member(const McOut &O, int32_t at, int32_t v, int32_t rec) {
  *(CG_GLOBAL i32x2 *)(O.tmp + 2 * (int64_t)at) = i32x2{v, rec};
}

// the tile-list slot of listed read v of local number l
__device__ __forceinline__ int32_t mc_list_slot(int32_t v, int32_t l, const int32_t *wp) {
  const int32_t t = v / kMaskTile;
  return t * kMaskTile + (l - wp[t * (kMaskTile / 32)]);
}

// component record cb: label, size, kind, first member slot; bases weight 0
__device__ __forceinline__ void mc_component(const McOut &O, int32_t cb, int32_t label,
                                             uint32_t c4, int32_t mb) {
  O.comp_label[cb] = label;
  O.comp_size[cb] = (int32_t)(c4 >> 2);
  O.comp_kind[cb] = kind_of(c4);
  O.memb[cb] = mb;
  O.comp_w[cb] = 0;
}

// local number of listed read v: listed reads before its word, plus those
// below it in the word
__device__ __forceinline__ int32_t mc_rank(const uint32_t *lw, const int32_t *wp, int32_t v) {
  const int w = v >> 5, b = v & 31;
  return wp[w] + __popc(lw[w] & ((1u << b) - 1u));
}

// id of the listed read of local number l (l below the number of listed
// reads; -1 otherwise)
__device__ __forceinline__ int32_t mc_select(const uint32_t *lw, const int32_t *wp, int W,
                                             int32_t l) {
  int lo = 0, hi = W - 1;  // the last word whose prefix is at most l holds it
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wp[mid] <= l) lo = mid;
    else hi = mid - 1;
  }
  uint32_t bits = lw[lo];
  for (int s = l - wp[lo]; s > 0 && bits; --s) bits &= bits - 1u;
  return bits ? (lo << 5) + __builtin_ctz(bits) : -1;
}

// State of the listed reads as the sweep over all reads sees it: entry
// (id | kept bits << 30), root (~component once numbered) and counter
// (per-root count, then member cursor).
template <bool kLds>
struct McState;
template <>
struct McState<true> {
  uint32_t *lid;
  int32_t *par;
  int32_t *cnt;
};
template <>
struct McState<false> {
  CG_GLOBAL uint32_t *lid;
  CG_GLOBAL int32_t *par;
  CG_GLOBAL int32_t *cnt;
};

// The outputs of one read of a job for phase H (and, with one-read
// components eligible, what numbering it needs): every LDS access happens
// whatever the read is (indices stay in range), so the loads of a thread's
// reads are issued together.
struct McRead {
  uint32_t fl;      // flags
  int32_t lab;      // label
  int32_t lcx;      // label_comp (-1 unless an eligible root already numbered)
  int32_t loc;      // local number of a read with kept entries, else -1
  int32_t root;     // root (local number) of a read with kept entries not yet numbered, else -1
  uint32_t c4;      // what an unnumbered root counts (4 per read + path ends); 4 for one read
  bool cand;        // not a branch read, not a member below a root: a component of its own
};

template <bool kLds>
__device__ __forceinline__ McRead mc_read(int32_t v, int32_t n, uint32_t lw, uint32_t bw,
                                          int32_t wp, const McState<kLds> &S) {
  McRead r;
  const int b = v & 31;
  const bool live = v < n;
  const bool listed = live && ((lw >> b) & 1u);
  const uint32_t br = live ? (bw >> b) & 1u : 0u;
  const int32_t l = listed ? wp + __popc(lw & ((1u << b) - 1u)) : 0;
  const uint32_t x = S.lid[l];
  const int32_t p = S.par[l];
  const uint32_t c = (uint32_t)S.cnt[l];
  const uint32_t y = S.lid[p >= 0 ? p : l];
  const uint32_t kept = listed ? x >> 30 : 0u;
  r.fl = br | (kept << 1);
  r.lab = v;
  r.lcx = -1;
  r.loc = kept ? l : -1;
  r.root = -1;
  r.c4 = 4;
  r.cand = live && !br;
  if (kept) {
    if (p >= 0 && p != l) {  // a member: its root comes earlier in id order
      r.root = p;
      r.lab = (int32_t)(y & kIdMask);
      r.cand = false;
    } else if (p < 0) {      // a root numbered by the listed scan
      r.lcx = ~p;
      r.cand = false;
    } else {                 // a root not numbered yet
      r.root = l;
      r.c4 = c;
    }
  }
  return r;
}

__device__ __forceinline__ void mc_store4(const McOut &O, int32_t v4, int32_t n, const McRead *r) {
  if (v4 + 3 < n) {
    *(CG_GLOBAL uint32_t *)(O.flags + v4) =
        r[0].fl | (r[1].fl << 8) | (r[2].fl << 16) | (r[3].fl << 24);
    *(CG_GLOBAL i32x4 *)(O.label + v4) = i32x4{r[0].lab, r[1].lab, r[2].lab, r[3].lab};
    *(CG_GLOBAL i32x4 *)(O.label_comp + v4) = i32x4{r[0].lcx, r[1].lcx, r[2].lcx, r[3].lcx};
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (v4 + i < n) {
        O.flags[v4 + i] = (uint8_t)r[i].fl;
        O.label[v4 + i] = r[i].lab;
        O.label_comp[v4 + i] = r[i].lcx;
      }
  }
}

// F when one-read components are eligible, with H: every read in id order,
// 4096 per round; the eligible components are numbered in label order
// (one-read components included) and members claim their slots.
template <bool kLds>
__device__ __forceinline__ int32_t mc_sweep_table(int32_t n, int32_t min_reads, const McOut &O,
                                                  const uint32_t *lw, const uint32_t *bw,
                                                  const int32_t *wp, const McState<kLds> &S,
                                                  int64_t *sh64) {
  const int32_t mr = min_reads < 1 ? 1 : min_reads;
  int32_t cbase = 0, mbase = 0;
  for (int32_t base = 0; base < n; base += 4 * kMcBlock) {
    const int32_t v4 = base + 4 * (int32_t)threadIdx.x;
    const int w = v4 < n ? v4 >> 5 : 0;
    McRead r[4];
    int64_t cnt = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      r[i] = mc_read<kLds>(v4 + i, n, lw[w], bw[w], wp[w], S);
      if (r[i].cand && (int32_t)(r[i].c4 >> 2) >= mr)
        cnt += ((int64_t)1 << 32) | (int64_t)(r[i].c4 >> 2);
      else
        r[i].cand = false;
    }
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, kMcBlock>(cnt, sh64, &tot);
    int32_t cb = cbase + (int32_t)(ex >> 32), mb = mbase + (int32_t)(ex & 0xFFFFFFFF);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!r[i].cand) continue;
      const int32_t v = v4 + i;
      mc_component(O, cb, v, r[i].c4, mb);
      r[i].lcx = cb;
      if (r[i].loc >= 0) {
        S.par[r[i].loc] = ~cb;
        S.cnt[r[i].loc] = mb;  // member cursor, the root's own slot included
      } else {
        mc_member(O, mb, v, kNoSlot);  // a one-read component is its own member
      }
      ++cb;
      mb += (int32_t)(r[i].c4 >> 2);
    }
    cbase += (int32_t)(tot >> 32);
    mbase += (int32_t)(tot & 0xFFFFFFFF);
    if (kLds) lds_barrier();
    else __syncthreads();
    // members (the roots of this round included) claim their slots
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (r[i].root < 0) continue;
      int32_t at;
      if constexpr (kLds) at = atomicAdd(S.cnt + r[i].root, 1);
      else at = mc_add(S.cnt + r[i].root, 1);
      if (at >= 0)
        mc_member(O, at, v4 + i,
                  kLds ? mc_list_slot(v4 + i, r[i].loc, wp) | (int32_t)((r[i].fl >> 1) << 30)
                       : kNoSlot);
    }
    if (v4 < n) mc_store4(O, v4, n, r);
  }
  return cbase;
}

// H (for jobs whose listed reads are in LDS, after F and G): what the
// listed reads change of the defaults the tile pass stored (the branch bit,
// own id, -1): kept bits, a member's label (its root's id), a numbered
// root's component.  Scattered stores of the listed reads only; all loads of
// the kernel are done by now (gfx9 counts stores and loads in one counter,
// so a load behind these stores would wait for them).
__device__ __forceinline__ void mc_write_listed(int32_t L, const McOut &O, const uint32_t *s_lid,
                                                const int32_t *s_b) {
  for (int32_t l = threadIdx.x; l < L; l += kMcBlock) {
    const uint32_t x = s_lid[l];
    const uint32_t kept = x >> 30;
    if (!kept) continue;
    const int32_t v = (int32_t)(x & kIdMask);
    const int32_t rt = s_b[l];
    O.flags[v] = (uint8_t)(kept << 1);
    if (rt < 0) O.label_comp[v] = ~rt;
    else if (rt != l) O.label[v] = (int32_t)(s_lid[rt] & kIdMask);
  }
}

// C-H for a job with more listed reads than LDS holds: the listed reads
// [lo, hi) of this thread (those of its words [w0, w1)) with their state in
// the job's scratch.  Returns the job's component count.
template <bool kLds>
__device__ __forceinline__ int32_t mc_components(
    const BJob &J, const McOut &O, const McArr<kLds> &A, const uint32_t *lw, const uint32_t *bw,
    const int32_t *wp, int32_t w0, int32_t w1, int32_t lo, int32_t hi, int64_t *sh64,
    int32_t *s_ml) {
  const int32_t n = J.g.n;
  const CG_GLOBAL int32_t *rp = (const CG_GLOBAL int32_t *)J.g.row_ptr;
  const CG_GLOBAL int32_t *col = (const CG_GLOBAL int32_t *)J.g.col;
  auto barrier = [] {
    if (kLds) lds_barrier();
    else __syncthreads();
  };
  // C. entries of each listed read: kept bits, first pointer, hook
  {
    int32_t m_l = 0;
    int32_t l = lo;  // this thread's listed reads, in order, by walking its words' bits
    for (int32_t w = w0; w < w1; ++w) {
      for (uint32_t bits = lw[w]; bits; bits &= bits - 1u, ++l) {
        const int32_t v = (w << 5) + __builtin_ctz(bits);
        const int32_t ra = rp[v], d = rp[v + 1] - ra;  // d is 1 or 2
        const int32_t c0 = col[ra], c1 = d == 2 ? col[ra + 1] : -1;
        uint32_t kept = 0;
        int32_t nb[2] = {-1, -1};
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int32_t c = j ? c1 : c0;
          if (c < 0) continue;
          const int cw = c >> 5, cb = c & 31;
          // kept: the other end is not a branch read (on a valid graph it is
          // then listed, which its local number needs; checked all the same)
          if (((bw[cw] >> cb) & 1u) || !((lw[cw] >> cb) & 1u)) continue;
          kept |= 1u << j;
          nb[j] = wp[cw] + __popc(lw[cw] & ((1u << cb) - 1u));
        }
        const int32_t s0 = nb[0] >= 0 && nb[0] < l ? nb[0] : l;
        const int32_t s1 = nb[1] >= 0 && nb[1] < l ? nb[1] : l;
        A.lid[l] = (uint32_t)v | (kept << 30);
        A.a[l] = s0 < s1 ? s0 : s1;                                // first pointer
        A.b[l] = (s0 < l && s1 < l) ? (s0 < s1 ? s1 : s0) : -1;  // the edge it leaves open
        m_l += __popc(kept);
      }
    }
    const int32_t wm = (int32_t)wave_sum((int64_t)m_l);
    if (lane_id() == 0 && wm) atomicAdd(s_ml, wm);
  }
  barrier();
  // D. hooks
  for (int32_t l = lo; l < hi; ++l) {
    const int32_t o = A.b[l];
    if (o >= 0) mc_union(A.a, l, o);
  }
  barrier();
  // E. roots, then per-root counts
  for (int32_t l = lo; l < hi; ++l) A.b[l] = (A.lid[l] >> 30) ? mc_find(A.a, l) : l;
  barrier();
  for (int32_t l = lo; l < hi; ++l) A.a[l] = 0;
  barrier();
  for (int32_t l = lo; l < hi; ++l) {
    const uint32_t kept = A.lid[l] >> 30;
    if (kept) mc_add(A.a + A.b[l], 4 + (__popc(kept) == 1 ? 1 : 0));
  }
  barrier();
  // H. every read's flags, label and label_comp hold their defaults (the
  // branch bit, own id, -1) from the tile pass; F and G store the changes
  // F. eligible components in label order, numbered from the threads' runs
  // (one scan), member cursors in `a`, ~component in `b` of a numbered root
  int32_t n_comp;
  if (J.min_reads >= 2) {
    int64_t cnt = 0;
    for (int32_t l = lo; l < hi; ++l)
      if ((A.lid[l] >> 30) && A.b[l] == l && (A.a[l] >> 2) >= J.min_reads)
        cnt += ((int64_t)1 << 32) | (int64_t)(A.a[l] >> 2);
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, kMcBlock>(cnt, sh64, &tot);
    int32_t cb = (int32_t)(ex >> 32), mb = (int32_t)(ex & 0xFFFFFFFF);
    for (int32_t l = lo; l < hi; ++l) {
      if (!(A.lid[l] >> 30) || A.b[l] != l) continue;
      const uint32_t c4 = (uint32_t)A.a[l];
      if ((int32_t)(c4 >> 2) >= J.min_reads) {
        mc_component(O, cb, (int32_t)(A.lid[l] & kIdMask), c4, mb);
        A.b[l] = ~cb;
        A.a[l] = mb;
        ++cb;
        mb += (int32_t)(c4 >> 2);
      } else {
        A.a[l] = kNotEligible;
      }
    }
    n_comp = (int32_t)(tot >> 32);
  } else {
    // one-read components are eligible too: every read that is not a branch
    // read and not a member below a root is a component of its own
    const int32_t mr = J.min_reads < 1 ? 1 : J.min_reads;  // at most 1 here
    uint32_t sm[kMcMaxWpt], rm[kMcMaxWpt];  // one-read and root masks of each word
    int64_t cnt = 0;
    {
      int32_t l = lo;
#pragma unroll
      for (int k = 0; k < kMcMaxWpt; ++k) {
        const int32_t w = w0 + k;
        sm[k] = rm[k] = 0;
        if (w >= w1) continue;
        const int32_t v0 = w << 5;
        const uint32_t valid = v0 + 32 <= n ? ~0u : ((1u << (n - v0)) - 1u);
        sm[k] = valid & ~bw[w] & ~lw[w];
        for (uint32_t bits = lw[w]; bits; bits &= bits - 1u, ++l) {
          const uint32_t bit = bits & (0u - bits);
          if (!(A.lid[l] >> 30)) {
            sm[k] |= bit;
          } else if (A.b[l] == l && (A.a[l] >> 2) >= mr) {
            rm[k] |= bit;
            cnt += (int64_t)(A.a[l] >> 2) - 1;  // the root's reads beyond one
          }
        }
        cnt += (int64_t)__popc(sm[k] | rm[k]) * (((int64_t)1 << 32) | 1);
      }
    }
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, kMcBlock>(cnt, sh64, &tot);
    int32_t cb = (int32_t)(ex >> 32), mb = (int32_t)(ex & 0xFFFFFFFF);
    int32_t l = lo;
#pragma unroll
    for (int k = 0; k < kMcMaxWpt; ++k) {
      const int32_t w = w0 + k;
      if (w >= w1) continue;
      const int32_t v0 = w << 5;
      const uint32_t lwk = lw[w];
      for (uint32_t bits = sm[k] | rm[k]; bits; bits &= bits - 1u) {
        const int b = __builtin_ctz(bits);
        const int32_t v = v0 + b;
        uint32_t c4 = 4;
        if ((rm[k] >> b) & 1u) {
          const int32_t lr = l + __popc(lwk & ((1u << b) - 1u));
          c4 = (uint32_t)A.a[lr];
          A.b[lr] = ~cb;
          A.a[lr] = mb;  // member cursor, the root's own slot included
        } else {
          mc_member(O, mb, v, kNoSlot);  // a one-read component is its own member
        }
        mc_component(O, cb, v, c4, mb);
        O.label_comp[v] = cb;
        ++cb;
        mb += (int32_t)(c4 >> 2);
      }
      l += __popc(lwk);
    }
    n_comp = (int32_t)(tot >> 32);
  }
  barrier();
  // G. members claim their slots; what the listed reads change in H's
  // stores: kept bits, a member's label, a numbered root's label_comp
  for (int32_t l = lo; l < hi; ++l) {
    const uint32_t x = A.lid[l];
    const uint32_t kept = x >> 30;
    if (!kept) continue;
    const int32_t v = (int32_t)(x & kIdMask);
    const int32_t rt = A.b[l];
    const int32_t r = rt < 0 ? l : rt;
    const int32_t at = mc_add(A.a + r, 1);
    if (at >= 0) mc_member(O, at, v, kNoSlot);
    O.flags[v] = (uint8_t)(kept << 1);
    if (rt < 0) O.label_comp[v] = ~rt;
    else if (rt != l) O.label[v] = (int32_t)(A.lid[rt] & kIdMask);
  }
  return n_comp;
}

// C-G for the listed reads of this thread, their state in LDS: slot k holds
// local number tid + k * kMcBlock (below L), so that the slots' loads of the
// tile lists are contiguous across a wave; PER is the listed reads per thread
// rounded up to 1, 2, 4 or kMcPer, so that a job does the work of its own
// reads.  Returns the job's component count (eligible components at
// min_reads >= 2; otherwise they are numbered by the sweep over all reads).
template <int PER>
__device__ __forceinline__ int32_t mc_listed(const BJob &J, const McOut &O, int32_t L,
                                             int32_t W, const uint32_t *lw, const uint32_t *bw,
                                             const int32_t *wp, uint32_t *s_lid, int32_t *s_a,
                                             int32_t *s_b, int64_t *sh64, int32_t *s_ml) {
  const int tid = threadIdx.x;
  int32_t ls[PER];  // local number of slot k, or -1
#pragma unroll
  for (int k = 0; k < PER; ++k) ls[k] = tid + k * kMcBlock < L ? tid + k * kMcBlock : -1;
  // C. each read's id and columns from its tile's list (tile t's listed
  // reads hold local numbers from the prefix of its first word on), then
  // kept bits and the other ends' local numbers from the bitmaps
  int32_t id[PER], c0[PER], c1[PER];
  int32_t slot[PER];
  {
    constexpr int kTileWords = kMaskTile / 32;
    const int32_t nt = J.mt_count;
    const CG_GLOBAL i32x4 *list = (const CG_GLOBAL i32x4 *)J.s.walk;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int32_t l = ls[k] >= 0 ? ls[k] : 0;
      int32_t a = 0, b = nt - 1;  // the last tile whose first local number is at most l
      while (a < b) {
        const int32_t mid = (a + b + 1) >> 1;
        if (wp[mid * kTileWords] <= l) a = mid;
        else b = mid - 1;
      }
      slot[k] = a * kMaskTile + (l - wp[a * kTileWords]);
    }
    i32x4 e[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) e[k] = list[slot[k]];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      id[k] = ls[k] >= 0 ? e[k].x : -1;
      c0[k] = ls[k] >= 0 ? e[k].y : -1;
      c1[k] = ls[k] >= 0 ? e[k].z : -1;
    }
  }
  uint32_t kept[PER];
  int32_t hook[PER];
  {
    int32_t m_l = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int32_t l = ls[k];
      // kept: the other end is not a branch read (on a valid graph it is
      // then listed, which its local number needs; checked all the same)
      const int32_t x0 = c0[k] >= 0 ? c0[k] : 0, x1 = c1[k] >= 0 ? c1[k] : 0;
      const uint32_t b0 = bw[x0 >> 5], b1 = bw[x1 >> 5];
      const uint32_t w0 = lw[x0 >> 5], w1 = lw[x1 >> 5];
      const int32_t f0 = wp[x0 >> 5], f1 = wp[x1 >> 5];
      const bool k0 = c0[k] >= 0 && !((b0 >> (x0 & 31)) & 1u) && ((w0 >> (x0 & 31)) & 1u);
      const bool k1 = c1[k] >= 0 && !((b1 >> (x1 & 31)) & 1u) && ((w1 >> (x1 & 31)) & 1u);
      kept[k] = (k0 ? 1u : 0u) | (k1 ? 2u : 0u);
      const int32_t n0 = k0 ? f0 + __popc(w0 & ((1u << (x0 & 31)) - 1u)) : l;
      const int32_t n1 = k1 ? f1 + __popc(w1 & ((1u << (x1 & 31)) - 1u)) : l;
      const int32_t s0 = n0 < l ? n0 : l, s1 = n1 < l ? n1 : l;
      // first pointer: the smallest kept neighbour below l; the edge to the
      // other one, when both lie below, is the hook left open
      hook[k] = (s0 < l && s1 < l) ? (s0 < s1 ? s1 : s0) : -1;
      if (l < 0) continue;
      s_lid[l] = (uint32_t)id[k] | (kept[k] << 30);
      s_a[l] = s0 < s1 ? s0 : s1;
      m_l += __popc(kept[k]);
    }
    const int32_t wm = (int32_t)wave_sum((int64_t)m_l);
    if (lane_id() == 0 && wm) atomicAdd(s_ml, wm);
  }
  lds_barrier();
  // D. hooks, one after the other
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (hook[k] >= 0) mc_union(s_a, ls[k], hook[k]);
  lds_barrier();
  // E. roots (lockstep climbs), then per-root counts
  int32_t r[PER];
  {
#pragma unroll
    for (int k = 0; k < PER; ++k) r[k] = ls[k] >= 0 ? ls[k] : 0;
    bool more = true;
    while (more) {
      more = false;
      int32_t pr[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        pr[k] = mc_ld(s_a + r[k]);
        if (!kept[k]) pr[k] = r[k];
      }
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        if (pr[k] != r[k]) more = true;
        r[k] = pr[k];
      }
    }
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (ls[k] < 0) continue;
    s_b[ls[k]] = r[k];
    s_a[ls[k]] = 0;
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (kept[k]) atomicAdd(s_a + r[k], 4 + (__popc(kept[k]) == 1 ? 1 : 0));
  lds_barrier();
  if (J.min_reads < 2) return 0;  // numbered by the sweep over all reads
  // F. eligible roots in label order: each thread numbers a contiguous run of
  // local numbers (which follow ids), one scan
  const int per = (L + kMcBlock - 1) / kMcBlock;
  const int32_t f0 = tid * per < L ? tid * per : L;
  const int32_t f1 = f0 + per < L ? f0 + per : L;
  int64_t c = 0;
  for (int32_t l = f0; l < f1; ++l)
    if ((s_lid[l] >> 30) && s_b[l] == l && (s_a[l] >> 2) >= J.min_reads)
      c += ((int64_t)1 << 32) | (int64_t)(s_a[l] >> 2);
  int64_t tot;
  const int64_t ex = block_excl_scan<int64_t, kMcBlock>(c, sh64, &tot);
  int32_t cb = (int32_t)(ex >> 32), mb = (int32_t)(ex & 0xFFFFFFFF);
  for (int32_t l = f0; l < f1; ++l) {
    if (!(s_lid[l] >> 30) || s_b[l] != l) continue;
    const uint32_t c4 = (uint32_t)s_a[l];
    if ((int32_t)(c4 >> 2) >= J.min_reads) {
      mc_component(O, cb, (int32_t)(s_lid[l] & kIdMask), c4, mb);
      s_b[l] = ~cb;
      s_a[l] = mb;  // member cursor, the root's own slot included
      ++cb;
      mb += (int32_t)(c4 >> 2);
    } else {
      s_a[l] = kNotEligible;
    }
  }
  lds_barrier();
  // G. members claim their slots
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (!kept[k]) continue;
    const int32_t at = atomicAdd(s_a + r[k], 1);
    if (at >= 0) mc_member(O, at, id[k], slot[k] | (int32_t)(kept[k] << 30));
  }
  return (int32_t)(tot >> 32);
}

__global__ __launch_bounds__(kMcBlock) void kb_mask_cc(BatchDev B) {
  __shared__ uint32_t s_lw[kMcWords], s_bw[kMcWords];
  __shared__ int32_t s_wp[kMcWords];
  __shared__ uint32_t s_lid[kMcListCap];
  __shared__ int32_t s_a[kMcListCap], s_b[kMcListCap];
  __shared__ int64_t sh64[kMcBlock / kWave + 1];
  __shared__ int32_t s_ml;  // kept directed entries of the job
  const int j = ld_const(B.job_order, blockIdx.x);
  const BJob J = job_at(B.jobs, j);
  if (J.external) return;
  const int32_t n = J.g.n;
  if (n > kMcReadCap) return;  // such a job is external (set when the batch is made)
  const int tid = threadIdx.x;
  const McOut O = mc_out(J);
  const int32_t W = (n + 31) >> 5;
  const int32_t wpt = (W + kMcBlock - 1) / kMcBlock;  // at most kMcMaxWpt
  const int32_t w0 = tid * wpt < W ? tid * wpt : W;
  const int32_t w1 = w0 + wpt < W ? w0 + wpt : W;
  if (tid == 0) s_ml = 0;
  // A. the job's bitmaps (written by kb_mask_tiles) into LDS
  {
    const CG_GLOBAL uint32_t *bits = (const CG_GLOBAL uint32_t *)J.s.fill;
    for (int32_t w = tid; w < W; w += kMcBlock) {
      s_lw[w] = bits[w];
      s_bw[w] = bits[W + w];
    }
  }
  __syncthreads();
  // B. listed reads before each word, and the branch reads of the job
  int32_t lo, hi, L, n_branch;
  {
    int64_t x = 0;
    for (int32_t w = w0; w < w1; ++w)
      x += ((int64_t)__popc(s_lw[w]) << 32) | (int64_t)__popc(s_bw[w]);
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, kMcBlock>(x, sh64, &tot);
    lo = (int32_t)(ex >> 32);
    hi = lo + (int32_t)(x >> 32);
    int32_t run = lo;
    for (int32_t w = w0; w < w1; ++w) {
      s_wp[w] = run;
      run += __popc(s_lw[w]);
    }
    L = (int32_t)(tot >> 32);
    n_branch = (int32_t)(tot & 0xFFFFFFFF);
  }
  lds_barrier();
  int32_t n_comp = 0;
  if (L <= kMcListCap) {
    const bool table = J.min_reads < 2;
    if (L > 0) {
      const int per = (L + kMcBlock - 1) / kMcBlock;
      if (per <= 1)
        n_comp = mc_listed<1>(J, O, L, W, s_lw, s_bw, s_wp, s_lid, s_a, s_b, sh64, &s_ml);
      else if (per <= 2)
        n_comp = mc_listed<2>(J, O, L, W, s_lw, s_bw, s_wp, s_lid, s_a, s_b, sh64, &s_ml);
      else if (per <= 4)
        n_comp = mc_listed<4>(J, O, L, W, s_lw, s_bw, s_wp, s_lid, s_a, s_b, sh64, &s_ml);
      else
        n_comp = mc_listed<kMcPer>(J, O, L, W, s_lw, s_bw, s_wp, s_lid, s_a, s_b, sh64, &s_ml);
    }
    if (table)
      n_comp = mc_sweep_table<true>(n, J.min_reads, O, s_lw, s_bw, s_wp,
                                    McState<true>{s_lid, s_b, s_a}, sh64);
    else
      mc_write_listed(L, O, s_lid, s_b);
  } else {
    n_comp = mc_components<false>(J, O,
                                  McArr<false>{(CG_GLOBAL uint32_t *)J.s.lidx,
                                               (CG_GLOBAL int32_t *)J.s.aux,
                                               (CG_GLOBAL int32_t *)J.s.walk},
                                  s_lw, s_bw, s_wp, w0, w1, lo, hi, sh64, &s_ml);
  }
  // BranchRemoval's counts (the kept entries were summed in LDS before the
  // later barriers) and the number of components; no barrier waits here for
  // the stores above
  if (tid == 0) {
    CG_GLOBAL int32_t *counts = (CG_GLOBAL int32_t *)J.counts;
    counts[0] = n_branch;
    counts[1] = s_ml;
    *(CG_GLOBAL int32_t *)J.parts.d_n_comp = n_comp;
  }
}

// 3b. bases weight of each eligible component (jobs partitioned by bases):
// the lengths of its reads, added at the component's entry
template <int T>
__global__ __launch_bounds__(T) void kb_weight(BatchDev B) {
  const int t = blockIdx.x;
  const BJob J = job_at(B.jobs, ld_const(B.tile_job, t));
  if (J.weight != CG_WEIGHT_BASES || J.external) return;
  const int64_t v = (int64_t)(t - J.vt_first) * T + threadIdx.x;
  if (v >= J.g.n) return;
  const int32_t c = J.parts.label_comp[J.label[v]];
  if (c >= 0) atomicAdd((unsigned long long *)J.s.comp_w + c, (unsigned long long)J.g.read_len[v]);
}

// 4. LPT per job (one workgroup each), bin offsets, bucket cursors; the last
// workgroup lays out the batch-wide component and piece item ranges
// the batched form's LPT runs one job per workgroup of 256 threads, so that
// all jobs' workgroups are resident at once
constexpr int kBatchLptBlock = 256;
// pieces per copy chunk (one wave each).  Chunks are handed to waves as
// slots free up, so the copy ends with a tail of the last chunks: 64 pieces
// (about 75 us of one wave's work on 3 kbp pieces) left it long, 16 paid the
// per-chunk setup too often.  The jobs holding the last sixteenth of the
// batch's pieces (the last chunks handed out, about one per wave slot) take
// chunks of kTailChunkPieces, so the waves that start last finish sooner.
constexpr int kChunkPieces = 32;
constexpr int kTailChunkPieces = 8;
constexpr int kWqBuckets = 4096;  // read counts from kWqBuckets - 1 up share the top bucket
constexpr int kBatchSortCap = 2048;
constexpr int kBatchBinCap = 256;

__global__ __launch_bounds__(kBatchLptBlock) void kb_lpt(BatchDev B) {
  __shared__ uint64_t s_keys[kBatchSortCap];
  __shared__ int32_t s_bin[kBatchSortCap];
  __shared__ uint64_t s_binA[kBatchBinCap], s_binB[kBatchBinCap];
  __shared__ int64_t sh[kBatchLptBlock / kWave + 1];
  const int j = blockIdx.x;
  const BJob J = job_at(B.jobs, j);
  const int P = J.P;
  const int nc = *J.parts.d_n_comp;
  const uint64_t *wts = J.weight == CG_WEIGHT_BASES ? J.s.comp_w : nullptr;
  const bool ext = J.external != 0;
  int m_e = 0;
  int64_t carry = 0;
  // the work-queue buckets start from zero for kb_tables / kb_wq_place
  for (int b = j * kBatchLptBlock + (int)threadIdx.x; b < kWqBuckets; b += (int)gridDim.x * kBatchLptBlock) {
    B.wq_hist[b] = 0;
    B.wq_cur[b] = 0;
  }
  if (!ext) {
    if (nc <= kBatchSortCap && P <= kBatchBinCap)
      m_e = lpt_body<kBatchLptBlock>(nc, P, J.parts.comp_size, wts, s_keys, s_bin, s_binA, s_binB, J.parts.comp_bin,
                     J.parts.comp_rank, J.parts.comp_start, J.parts.bin_load, J.s.bin_reads,
                     &B.fixed->status, J.parts.comp_kind, J.s.estart);
    else
      m_e = lpt_body<kBatchLptBlock>(nc, P, J.parts.comp_size, wts, J.s.keys, J.s.aux, J.s.bins, J.s.bins + P,
                     J.parts.comp_bin, J.parts.comp_rank, J.parts.comp_start, J.parts.bin_load,
                     J.s.bin_reads, &B.fixed->status, J.parts.comp_kind, J.s.estart);
    __syncthreads();
    // bin boundaries: prefix of the reads of each bin
    for (int base = 0; base < P; base += kBatchLptBlock) {
      const int b = base + threadIdx.x;
      const int64_t x = b < P ? (int64_t)__hip_atomic_load(J.s.bin_reads + b, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)
                              : 0;
      int64_t tot;
      const int64_t ex = block_excl_scan<int64_t, kBatchLptBlock>(x, sh, &tot);
      if (b < P) J.local.bin_vptr[b] = (int32_t)(carry + ex);
      carry += tot;
    }
  }
  __shared__ int last;
  if (threadIdx.x == 0) {
    if (!ext) {
      J.local.bin_vptr[P] = (int32_t)carry;
      J.local.d_sizes[0] = (int32_t)carry;
      J.local.d_sizes[1] = m_e;
      J.local.loc_row_ptr[carry] = m_e;
    }
    // dense, for the last workgroup; an external job adds no components or
    // pieces to the batch-wide queues
    B.job_cnt[j] = ext ? make_int2(0, 0) : make_int2(nc, (int32_t)carry);
    __threadfence();
    last = atomicAdd(&B.counters[2], 1u) == (unsigned)B.n_jobs - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  // each thread sums a run of consecutive jobs; two scans give the bases:
  // (components << 32) | pieces (each total below 2^31) and chunks
  const int per = (B.n_jobs + kBatchLptBlock - 1) / kBatchLptBlock;
  const int i0 = (int)threadIdx.x * per;
  const int i1 = i0 + per < B.n_jobs ? i0 + per : B.n_jobs;
  int64_t xcp = 0, xh = 0;
  for (int i = i0; i < i1; ++i) {
    const uint64_t w = __hip_atomic_load((uint64_t *)(B.job_cnt + i), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    const int64_t xc = (int32_t)(uint32_t)w, xp = (int32_t)(uint32_t)(w >> 32);
    xcp += (xc << 32) | xp;
  }
  int64_t tcp, th;
  int64_t ecp = block_excl_scan<int64_t, kBatchLptBlock>(xcp, sh, &tcp);
  // chunks: a job whose pieces reach into the last sixteenth of the
  // batch's takes the tail chunk size
  const int64_t np = (int64_t)(uint32_t)tcp;
  const int64_t tail_at = np - (np >> 4);
  {
    int64_t pc = (int64_t)(uint32_t)ecp;
    for (int i = i0; i < i1; ++i) {
      const uint64_t w = __hip_atomic_load((uint64_t *)(B.job_cnt + i), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      const int64_t xp = (int32_t)(uint32_t)(w >> 32);
      const int cp = pc + xp > tail_at ? kTailChunkPieces : kChunkPieces;
      xh += (xp + cp - 1) / cp;
      pc += xp;
    }
  }
  int64_t eh = block_excl_scan<int64_t, kBatchLptBlock>(xh, sh, &th);
  for (int i = i0; i < i1; ++i) {
    const uint64_t w = __hip_atomic_load((uint64_t *)(B.job_cnt + i), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    const int64_t xc = (int32_t)(uint32_t)w, xp = (int32_t)(uint32_t)(w >> 32);
    const int cp = (int64_t)(uint32_t)ecp + xp > tail_at ? kTailChunkPieces : kChunkPieces;
    B.comp_base[i] = (int32_t)(ecp >> 32);
    B.piece_base[i] = (int32_t)(uint32_t)ecp;
    B.chunk_base[i] = (int32_t)eh;
    B.chunk_cp[i] = cp;
    ecp += (xc << 32) | xp;
    eh += (xp + cp - 1) / cp;
  }
  if (threadIdx.x == 0) {
    B.comp_base[B.n_jobs] = (int32_t)(tcp >> 32);
    B.piece_base[B.n_jobs] = (int32_t)(uint32_t)tcp;
    B.chunk_base[B.n_jobs] = (int32_t)th;
    B.counters[2] = 0;
  }
  __threadfence();
}

// 4b. the job of every batch-wide component, so that the work queue's
// placement finds it with one load, and the queue's histogram: one entry per
// thread, by binary search in the bases (staged in LDS up to kTablesJobCap
// jobs)
constexpr int kTablesBlock = 256;
constexpr int kTablesJobCap = 4096;

__global__ __launch_bounds__(kTablesBlock) void kb_tables(BatchDev B) {
  __shared__ int32_t s_cb[kTablesJobCap + 1];
  __shared__ int32_t s_hist[kWqBuckets];
  for (int b = threadIdx.x; b < kWqBuckets; b += kTablesBlock) s_hist[b] = 0;
  const int nj = B.n_jobs;
  const bool in_lds = nj <= kTablesJobCap;
  if (in_lds) {
    for (int i = threadIdx.x; i <= nj; i += kTablesBlock) s_cb[i] = B.comp_base[i];
  }
  __syncthreads();
  const int32_t tc = B.comp_base[nj];
  for (int32_t i = blockIdx.x * kTablesBlock + threadIdx.x; i < tc;
       i += gridDim.x * kTablesBlock) {
    const int j = job_of(in_lds ? s_cb : B.comp_base, nj, i);
    B.comp_job[i] = j;
    // the work queue's histogram: components per read count
    const int32_t q = B.jobs[j].parts.comp_size[i - (in_lds ? s_cb[j] : B.comp_base[j])];
    atomicAdd(s_hist + (q < kWqBuckets - 1 ? q : kWqBuckets - 1), 1);
  }
  // (counted in LDS: many components share a read count, and their global
  // atomics would queue on one address)
  __syncthreads();
  for (int b = threadIdx.x; b < kWqBuckets; b += kTablesBlock)
    if (s_hist[b]) atomicAdd(B.wq_hist + b, s_hist[b]);
}

// 4c. the work queue: every component of the batch in decreasing read count
// (within a bucket in any order), as (job, component, reads, first local
// number), and the queue heads of the per-component passes.  Handing the
// largest components out first to whichever workgroup is free is LPT list
// scheduling of the whole batch's components onto the workgroups.
// Components above kIwCap reads form the queue's head (two passes, arrays
// in scratch), those of at most kWalkSmallCap its tail (one wave each).
constexpr int kWqBlock = 256;
constexpr int kWalkTinyCap = 32;  // reads of the components the tiny pass takes
// Reads of the components that the one-pass workgroup form takes (its walk
// arrays in LDS).  Each such component's time is mostly latency (dependent
// gathers, barriers), about the same from 129 to 512 reads, so the pass
// wants every component on a workgroup of its own: LDS sized for 512 reads
// (and 2 members per thread) lets four workgroups share a compute unit,
// where LDS for 1024 held two, so that a batch with more components above
// 128 reads than two per compute unit took two rounds of them.  Larger
// components take the two-pass form.
constexpr int kIwCap = 512;
constexpr int kWqPer = kWqBuckets / kWqBlock;

__device__ __forceinline__ WqE wq_make(const BJob &J, int j, int32_t c, int32_t q) {
  return WqE{j, c, q, J.parts.comp_start[c], J.s.estart[c], J.parts.comp_rank[c],
             J.s.tmp + 2 * (int64_t)J.s.memb[c]};
}

__global__ __launch_bounds__(kWqBlock) void kb_wq_place(BatchDev B) {
  __shared__ int32_t s_start[kWqBuckets], s_cnt[kWqBuckets], s_base[kWqBuckets];
  __shared__ int32_t sh[kWqBlock / kWave + 1];
  // start of each bucket: the components in larger buckets (a scan from the
  // top bucket down; thread t holds buckets kWqBuckets-1-t*kWqPer ... down)
  int32_t h[kWqPer], loc = 0;
#pragma unroll
  for (int k = 0; k < kWqPer; ++k) {
    h[k] = __hip_atomic_load(B.wq_hist + (kWqBuckets - 1 - (threadIdx.x * kWqPer + k)),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    loc += h[k];
  }
  int32_t tot;
  int32_t run = block_excl_scan<int32_t, kWqBlock>(loc, sh, &tot);
#pragma unroll
  for (int k = 0; k < kWqPer; ++k) {
    s_start[kWqBuckets - 1 - (threadIdx.x * kWqPer + k)] = run;
    run += h[k];
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    B.wq_meta[0] = tot;
    B.wq_meta[1] = s_start[kWalkSmallCap];  // components above kWalkSmallCap reads
    B.wq_meta[2] = s_start[kIwCap];         // above kIwCap
    B.wq_meta[3] = s_start[kWalkTinyCap];   // above kWalkTinyCap
  }
  // this workgroup's components: a contiguous range; counted per bucket in
  // LDS, one reservation per bucket in the queue, placed by LDS cursors
  const int32_t tc = B.comp_base[B.n_jobs];
  const int32_t per = (tc + (int32_t)gridDim.x - 1) / (int32_t)gridDim.x;
  const int32_t i0 = (int32_t)blockIdx.x * per;
  const int32_t i1 = i0 + per < tc ? i0 + per : tc;
  for (int b = threadIdx.x; b < kWqBuckets; b += kWqBlock) s_cnt[b] = 0;
  __syncthreads();
  // the thread's first component is kept in registers for the placement
  // (with 128 workgroups of 256 threads, every component of a batch of up to
  // 32768 is a first one); later ones are loaded again there
  WqE first{-1, 0, 0, 0, 0, 0, nullptr};
  for (int32_t i = i0 + threadIdx.x; i < i1; i += kWqBlock) {
    const int j = B.comp_job[i];
    const int32_t c = i - B.comp_base[j];
    const BJob &J = B.jobs[j];
    const int32_t q = J.parts.comp_size[c];
    if (i == i0 + (int32_t)threadIdx.x) first = wq_make(J, j, c, q);
    atomicAdd(s_cnt + (q < kWqBuckets - 1 ? q : kWqBuckets - 1), 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kWqBuckets; b += kWqBlock) {
    const int32_t k = s_cnt[b];
    s_base[b] = k ? s_start[b] + atomicAdd(B.wq_cur + b, k) : 0;
    s_cnt[b] = 0;
  }
  __syncthreads();
  for (int32_t i = i0 + threadIdx.x; i < i1; i += kWqBlock) {
    WqE e = first;
    if (i != i0 + (int32_t)threadIdx.x) {
      const int j = B.comp_job[i];
      const int32_t c = i - B.comp_base[j];
      const BJob &J = B.jobs[j];
      e = wq_make(J, j, c, J.parts.comp_size[c]);
    }
    const int b = e.q < kWqBuckets - 1 ? e.q : kWqBuckets - 1;
    B.wq[s_base[b] + atomicAdd(s_cnt + b, 1)] = e;
  }
}

// The per-component passes take their part of the work queue [lo, hi) in a
// snake order over the grid: round r gives workgroup w entry r*W + w, or
// r*W + W-1-w on odd rounds.  The queue is in decreasing read count, so this
// deals the components out like LPT list scheduling, with no atomics.
// Returns the entry of round r, or -1 past the end.
__device__ __forceinline__ int32_t wq_entry(int32_t lo, int32_t hi, int32_t r) {
  const int32_t W = (int32_t)gridDim.x, w = (int32_t)blockIdx.x;
  const int64_t x = (int64_t)lo + (int64_t)r * W + ((r & 1) ? W - 1 - w : w);
  return x < hi ? (int32_t)x : -1;
}

// entry x (uniform): (job, component, reads, first local number)
__device__ __forceinline__ int4 wq_at(const BatchDev &B, int32_t x) {
  const CG_CONST uint64_t *p = (const CG_CONST uint64_t *)(B.wq + x);
  const uint64_t a = p[0], b = p[1];
  return make_int4((int)(uint32_t)a, (int)(uint32_t)(a >> 32), (int)(uint32_t)b,
                   (int)(uint32_t)(b >> 32));
}
// the whole entry x (uniform), by scalar loads
__device__ __forceinline__ WqE wq_get(const BatchDev &B, int32_t x) {
  WqE e;
  const CG_CONST uint64_t *p = (const CG_CONST uint64_t *)(B.wq + x);
  uint64_t *q = reinterpret_cast<uint64_t *>(&e);
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = p[k];
  return e;
}

// 6. induced subgraph of each component: sorted local numbers and local CSR
// rows
template <int BLOCK, int CAP>
__device__ __forceinline__ void induce_listed(const BatchDev &B, int4 d, int32_t *a,
                                              int32_t *sh_scan) {
  // d = (job, component, reads, first local number), uniform
  const int j = __builtin_amdgcn_readfirstlane(d.x), c = __builtin_amdgcn_readfirstlane(d.y);
  const int q = __builtin_amdgcn_readfirstlane(d.z), st = __builtin_amdgcn_readfirstlane(d.w);
  const BJob J = job_at(B.jobs, j);
  // member records are (id, list slot) pairs
  const int32_t *members = J.s.tmp + 2 * (int64_t)J.s.memb[c];
  induce_component<BLOCK, CAP, 2>(q, st, J.s.estart[c], members, J.flags, J.g.row_ptr, J.g.col,
                               J.local.perm, J.s.lidx, J.local.loc_row_ptr, J.local.loc_col,
                               J.local.loc_eid, a, sh_scan);
}

// 6-7. InducedSubgraph and LocalAssembly of one component of at most CAP
// reads in one pass.  Each member's id, kept entries and neighbours come
// from its member record and the tile list, which gathered them in id
// order (a record without a list slot takes them from the graph), then its
// read length and its entries' strand bits and overlaps (or coordinates)
// from the graph.  The local numbers follow
// the ids; every field goes into the walk's LDS arrays at its local number
// while perm and the local CSR rows are written out, so the walk reads
// nothing back.
__device__ __forceinline__ int32_t lds_lower_bound(const int32_t *a, int q, int32_t x) {
  int lo = 0, hi = q;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <int BLOCK, int CAP>
__device__ __forceinline__ void iw_component(const BJob &J, const WqE &e, WalkArrays w,
                                             uint32_t *sh_scan) {
  constexpr int R = CAP >= BLOCK ? CAP / BLOCK : 1;  // members per thread
  const int tid = threadIdx.x;
  const int q = e.q, st = e.st;
  const CG_GLOBAL i32x2 *mem = (const CG_GLOBAL i32x2 *)e.mem;
  const CG_GLOBAL i32x4 *la = (const CG_GLOBAL i32x4 *)J.s.walk;
  const CG_GLOBAL uint32_t *glen = (const CG_GLOBAL uint32_t *)J.g.read_len;
  const CG_GLOBAL uint64_t *goff = (const CG_GLOBAL uint64_t *)J.g.read_off;
  const CG_GLOBAL uint8_t *gstr = (const CG_GLOBAL uint8_t *)J.g.strand;
  const CG_GLOBAL uint32_t *gov = (const CG_GLOBAL uint32_t *)(J.g.pre ? J.g.pre : J.g.ovl);
  const CG_GLOBAL uint32_t *gpost = (const CG_GLOBAL uint32_t *)J.g.post;
  const bool coords = J.g.post != nullptr;
  // 1. member records, then their list entries A = (id, first column,
  // second column, first entry) and kept bits kb; a record without a list
  // slot takes them from the graph (flags give the kept entries)
  // Every lane loads (a lane past the component member 0's record, a record
  // without a slot list entry 0), so that each round's loads are issued
  // together, without branches
  int32_t v[R], rec[R], vl[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = tid + u * BLOCK;
    const i32x2 m = mem[i < q ? i : 0];
    vl[u] = m.x;
    v[u] = i < q ? m.x : 0x7FFFFFFF;
    rec[u] = i < q ? m.y : kNoSlot;
  }
  // list entries, and the read lengths and store offsets in the same round
  i32x4 A[R];
  uint32_t kb[R];
  i32x4 Bq[R];
  i32x2 Cq[R];
  uint64_t ro[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    // (a record without a slot gets its entry from the graph below)
    A[u] = la[rec[u] != kNoSlot ? rec[u] & kNoSlot : 0];
    const uint32_t len = glen[vl[u]];
    const uint64_t off = goff[vl[u]];
    kb[u] = (uint32_t)rec[u] >> 30;
    Bq[u] = i32x4{(int32_t)len, 0, 0, 0};
    Cq[u] = i32x2{0, 0};
    ro[u] = off;
  }
  // the contig record's label and bin, loaded now and stored at the end
  const CompRec cr = comp_rec(J.parts, e.c, e.rank);
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = tid + u * BLOCK;
    if (i < q && rec[u] == kNoSlot) {
      const int32_t x = v[u];
      kb[u] = ((uint32_t)J.flags[x] >> 1) & 3u;
      const int32_t b = J.g.row_ptr[x];
      A[u] = i32x4{x, -1, -1, b};
      if (kb[u] & 1u) A[u].y = J.g.col[b];
      if (kb[u] & 2u) A[u].z = J.g.col[b + 1];
    }
  }
  // then the kept entries' strand bits, overlaps (or pre) and post: Bq =
  // (length, ov of entry 0, ov of entry 1, strands), Cq = post of both
#pragma unroll
  for (int u = 0; u < R; ++u) {
    if (tid + u * BLOCK >= q) continue;
    const int32_t b = A[u].w;
    if (kb[u] & 1u) {
      Bq[u].y = (int32_t)gov[b];
      Bq[u].w = gstr[b];
      if (coords) Cq[u].x = (int32_t)gpost[b];
    }
    if (kb[u] & 2u) {
      Bq[u].z = (int32_t)gov[b + 1];
      Bq[u].w |= (int32_t)gstr[b + 1] << 8;
      if (coords) Cq[u].y = (int32_t)gpost[b + 1];
    }
  }
  // 2. local numbers: the ids in order in a (the walk's nxt array, unused
  // until its rays), each member's rank among them
  int32_t *a = w.nxt;
  int32_t rk[R];
  if constexpr (BLOCK == kWave) {
    // one wave: a rank is the number of smaller ids, counted over the lanes
#pragma unroll
    for (int u = 0; u < R; ++u) rk[u] = 0;
#pragma unroll
    for (int u2 = 0; u2 < R; ++u2) {
      const int cnt = q - u2 * kWave < kWave ? q - u2 * kWave : kWave;
      for (int l2 = 0; l2 < cnt; ++l2) {
        const int32_t x = __builtin_amdgcn_readlane(v[u2], l2);
#pragma unroll
        for (int u = 0; u < R; ++u) rk[u] += x < v[u] ? 1 : 0;
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u)
      if (tid + u * BLOCK < q) a[rk[u]] = v[u];
    lds_barrier();
  } else {
    int N2 = 1;
    while (N2 < q) N2 <<= 1;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = tid + u * BLOCK;
      if (i < N2) a[i] = i < q ? v[u] : 0x7FFFFFFF;
    }
    lds_barrier();
    // ids are non-negative and the padding is the largest int32, so their
    // order as uint32 is the same; the stages within 64 elements run in
    // registers (8 barriers for 512 ids instead of 45), and the barriers
    // order LDS only, so the gathers above stay in flight
    bitonic_sort<uint32_t, true>(reinterpret_cast<uint32_t *>(a), N2);
#pragma unroll
    for (int u = 0; u < R; ++u) rk[u] = tid + u * BLOCK < q ? lds_lower_bound(a, q, v[u]) : 0;
  }
  // 3. every member's fields at its local number: its kept entries in row
  // order (slot 0, then slot 1), neighbours as local numbers
#pragma unroll
  for (int u = 0; u < R; ++u) {
    if (tid + u * BLOCK >= q) continue;
    const int r = rk[u];
    // slot 0: the first kept entry (entry 0, else entry 1); slot 1: entry 1
    // when both are kept (selects, no indexed arrays)
    const bool k0 = kb[u] & 1u, k1 = (kb[u] & 2u) != 0u;
    const bool s0 = k0 || k1, s1 = k0 && k1;
    const uint32_t sw = (uint32_t)Bq[u].w;
    const int32_t e0 = k0 ? A[u].w : A[u].w + 1, n0 = k0 ? A[u].y : A[u].z;
    const uint32_t es0 = k0 ? (sw & 0xFFu) : ((sw >> 8) & 0xFFu);
    const uint32_t eo0 = (uint32_t)(k0 ? Bq[u].y : Bq[u].z);
    const uint32_t ep0 = (uint32_t)(k0 ? Cq[u].x : Cq[u].y);
    w.nb[2 * r] = s0 ? lds_lower_bound(a, q, n0) : -1;
    w.eid[2 * r] = s0 ? e0 : -1;
    w.es[2 * r] = (uint8_t)(s0 ? es0 : 0u);
    w.eo[2 * r] = s0 ? eo0 : 0u;
    w.ep[2 * r] = s0 ? ep0 : 0u;
    w.nb[2 * r + 1] = s1 ? lds_lower_bound(a, q, A[u].z) : -1;
    w.eid[2 * r + 1] = s1 ? A[u].w + 1 : -1;
    w.es[2 * r + 1] = (uint8_t)(s1 ? (sw >> 8) & 0xFFu : 0u);
    w.eo[2 * r + 1] = s1 ? (uint32_t)Bq[u].z : 0u;
    w.ep[2 * r + 1] = s1 ? (uint32_t)Cq[u].y : 0u;
    w.vid[r] = v[u];
    w.rlen[r] = (uint32_t)Bq[u].x;
    w.roff[r] = ro[u];
  }
  lds_barrier();
  // 4. perm and the local CSR rows, in local order
  CG_GLOBAL int32_t *perm = (CG_GLOBAL int32_t *)J.local.perm;
  CG_GLOBAL int32_t *lrp = (CG_GLOBAL int32_t *)J.local.loc_row_ptr;
  CG_GLOBAL int32_t *lcol = (CG_GLOBAL int32_t *)J.local.loc_col;
  CG_GLOBAL int32_t *leid = (CG_GLOBAL int32_t *)J.local.loc_eid;
  const int32_t estart = e.estart;
  int32_t carry = 0;
  for (int base = 0; base < q; base += BLOCK) {
    const int i = base + tid;
    int32_t n0 = -1, n1 = -1;
    if (i < q) {
      n0 = w.nb[2 * i];
      n1 = w.nb[2 * i + 1];
    }
    const int32_t deg = (n0 >= 0 ? 1 : 0) + (n1 >= 0 ? 1 : 0);
    int32_t tot;
    const int32_t ex = block_excl_scan<int32_t, BLOCK, true>(deg, (int32_t *)sh_scan, &tot);
    if (i < q) {
      const int32_t r0 = estart + carry + ex;
      perm[st + i] = a[i];
      lrp[st + i] = r0;
      if (n0 >= 0) {
        lcol[r0] = st + n0;
        leid[r0] = w.eid[2 * i];
      }
      if (n1 >= 0) {
        lcol[r0 + 1] = st + n1;
        leid[r0 + 1] = w.eid[2 * i + 1];
      }
    }
    carry += tot;
  }
  walk_chain<BLOCK, CAP, true>(cr, q, st, w, J.g, J.local.perm, J.out, J.s, sh_scan);
}

// 6a. components of at most kWalkTinyCap reads (the queue's tail): one wave
// each, both steps in one pass, with small LDS arrays so that many waves run
// at once
__global__ __launch_bounds__(kWalkSmallBlock) void kb_induce_walk_tiny(BatchDev B) {
  __shared__ int32_t s_nb[2 * kWalkTinyCap], s_eid[2 * kWalkTinyCap], s_nxt[2 * kWalkTinyCap],
      s_dist[2 * kWalkTinyCap], s_endv[2 * kWalkTinyCap], s_vid[kWalkTinyCap];
  __shared__ uint32_t s_rlen[kWalkTinyCap], s_eo[2 * kWalkTinyCap], s_ep[2 * kWalkTinyCap];
  __shared__ uint64_t s_roff[kWalkTinyCap];
  __shared__ uint8_t s_es[2 * kWalkTinyCap];
  __shared__ uint32_t sh_scan[kWalkSmallBlock / kWave + 1];
  const int32_t lo = ld_const(B.wq_meta, 3), hi = ld_const(B.wq_meta, 0);
  // each round's entry is fetched while the previous round's component runs
  int32_t x = wq_entry(lo, hi, 0);
  WqE nx{};
  if (x >= 0) nx = wq_get(B, x);
  for (int32_t r = 1; x >= 0; ++r) {
    const WqE e = nx;
    x = wq_entry(lo, hi, r);
    if (x >= 0) nx = wq_get(B, x);
    const BJob J = job_at(B.jobs, e.job);
    WalkArrays w{s_nb, s_eid, s_nxt, s_dist, s_endv, s_vid, s_rlen, s_roff, s_es, s_eo, s_ep};
    iw_component<kWalkSmallBlock, kWalkTinyCap>(J, e, w, sh_scan);
  }
}

// 6b. components of kWalkTinyCap + 1 .. kWalkSmallCap reads: one wave each
__global__ __launch_bounds__(kWalkSmallBlock) void kb_induce_walk_small(BatchDev B) {
  __shared__ int32_t s_nb[2 * kWalkSmallCap], s_eid[2 * kWalkSmallCap], s_nxt[2 * kWalkSmallCap],
      s_dist[2 * kWalkSmallCap], s_endv[2 * kWalkSmallCap], s_vid[kWalkSmallCap];
  __shared__ uint32_t s_rlen[kWalkSmallCap], s_eo[2 * kWalkSmallCap], s_ep[2 * kWalkSmallCap];
  __shared__ uint64_t s_roff[kWalkSmallCap];
  __shared__ uint8_t s_es[2 * kWalkSmallCap];
  __shared__ uint32_t sh_scan[kWalkSmallBlock / kWave + 1];
  const int32_t lo = ld_const(B.wq_meta, 1), hi = ld_const(B.wq_meta, 3);
  // each round's entry is fetched while the previous round's component runs
  int32_t x = wq_entry(lo, hi, 0);
  WqE nx{};
  if (x >= 0) nx = wq_get(B, x);
  for (int32_t r = 1; x >= 0; ++r) {
    const WqE e = nx;
    x = wq_entry(lo, hi, r);
    if (x >= 0) nx = wq_get(B, x);
    const BJob J = job_at(B.jobs, e.job);
    WalkArrays w{s_nb, s_eid, s_nxt, s_dist, s_endv, s_vid, s_rlen, s_roff, s_es, s_eo, s_ep};
    // one member per lane up to kWave reads (a uniform branch), two above
    if (e.q <= kWave) iw_component<kWalkSmallBlock, kWave>(J, e, w, sh_scan);
    else iw_component<kWalkSmallBlock, kWalkSmallCap>(J, e, w, sh_scan);
  }
}

// 6c. components of kWalkSmallCap + 1 .. kIwCap reads: one workgroup each,
// both steps in one pass; and, first (the queue's head, largest first), the
// induced subgraph of each component above kIwCap reads, with the block
// sort in LDS up to kIndLocalCap reads, else in scratch (its walk, whose
// arrays reuse the tile lists' memory, waits for the next launch)
static_assert(kIndBlock == kWalkBlock, "one workgroup shape for both components' steps");
static_assert(kIndLocalCap <= 2 * kIwCap, "the induce step's sort buffer is the walk's nxt array");
static_assert(kIwCap <= kWalkCap && kIwCap % kWalkBlock == 0, "whole members per thread");
__global__ __launch_bounds__(kWalkBlock) void kb_induce_walk(BatchDev B) {
  __shared__ int32_t s_nb[2 * kIwCap], s_eid[2 * kIwCap], s_nxt[2 * kIwCap],
      s_dist[2 * kIwCap], s_endv[2 * kIwCap], s_vid[kIwCap];
  __shared__ uint32_t s_rlen[kIwCap], s_eo[2 * kIwCap], s_ep[2 * kIwCap];
  __shared__ uint64_t s_roff[kIwCap];
  __shared__ uint8_t s_es[2 * kIwCap];
  __shared__ uint32_t sh_scan[kWalkBlock / kWave + 1];
  const int32_t hi = ld_const(B.wq_meta, 1);
  // each round's entry is fetched while the previous round's component runs
  int32_t x = wq_entry(0, hi, 0);
  WqE nx{};
  if (x >= 0) nx = wq_get(B, x);
  for (int32_t r = 1; x >= 0; ++r) {
    const WqE e = nx;
    x = wq_entry(0, hi, r);
    if (x >= 0) nx = wq_get(B, x);
    if (e.q > kIwCap) {
      __syncthreads();  // the previous round's LDS is free
      induce_listed<kIndBlock, kIndLocalCap>(B, make_int4(e.job, e.c, e.q, e.st), s_nxt,
                                             (int32_t *)sh_scan);
      __syncthreads();
      continue;
    }
    const BJob J = job_at(B.jobs, e.job);
    WalkArrays w{s_nb, s_eid, s_nxt, s_dist, s_endv, s_vid, s_rlen, s_roff, s_es, s_eo, s_ep};
    iw_component<kWalkBlock, kIwCap>(J, e, w, sh_scan);
  }
}

// 7. their walks, with the walk's arrays in scratch
__global__ __launch_bounds__(kWalkBlock) void kb_walk(BatchDev B) {
  __shared__ uint32_t sh_scan[kWalkBlock / kWave + 1];
  const int32_t hi = ld_const(B.wq_meta, 2);
  for (int32_t r = 0, x; (x = wq_entry(0, hi, r)) >= 0; ++r) {
    const int4 d = wq_at(B, x);
    const int c = d.y, q = d.z, st = d.w;
    const BJob J = job_at(B.jobs, d.x);
    const int64_t n = J.g.n;
    int32_t *gb = J.s.walk;
    WalkArrays w{gb + 2 * (int64_t)st, gb + 2 * n + 2 * (int64_t)st,
                 gb + 4 * n + 4 * (int64_t)st, gb + 8 * n + 4 * (int64_t)st,
                 gb + 12 * n + 4 * (int64_t)st};
    walk_component<kWalkBlock, kWalkCap, false>(c, q, st, w, J.g, J.parts, J.local.perm,
                                                J.local.loc_row_ptr, J.local.loc_col,
                                                J.local.loc_eid, J.out, J.s, nullptr, sh_scan);
  }
}

// 8. contig word offsets per job, and the descriptors of its copy chunks
__global__ __launch_bounds__(kScanBlock) void kb_offsets(BatchDev B) {
  __shared__ unsigned long long sh[kScanBlock / kWave + 1];
  const BJob J = job_at(B.jobs, blockIdx.x);
  if (J.external) return;  // its offsets come from the single-graph assemble step
  const int nc = *J.parts.d_n_comp;
  unsigned long long carry = 0;
  for (int base = 0; base < nc; base += kScanBlock) {
    const int k = base + threadIdx.x;
    const unsigned long long wds = k < nc ? (J.out.len[k] + 15) / 16 : 0;
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan<unsigned long long, kScanBlock>(wds, sh, &tot);
    if (k < nc) J.out.base_off[k] = 16 * (carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0) {
    *J.out.d_total_words = carry;
    if (carry > J.out.cap_words) atomicOr(&B.fixed->status, CG_STATUS_BASES_OVERFLOW);
  }
  // the job's copy chunks, each in one 16-byte descriptor, so that a copy
  // wave starts from one load (none of the job's bases is written when
  // they overflow its buffer)
  const int32_t j = blockIdx.x;
  const int32_t h0 = B.chunk_base[j], h1 = B.chunk_base[j + 1];
  const int32_t n_e = B.piece_base[j + 1] - B.piece_base[j];
  const int32_t cp = B.chunk_cp[j];
  const bool over = carry > J.out.cap_words;
  for (int32_t h = h0 + (int32_t)threadIdx.x; h < h1; h += kScanBlock) {
    const int32_t c0 = (h - h0) * cp;
    const int32_t cnt = n_e - c0 < cp ? n_e - c0 : cp;
    B.chunk_desc[h] = make_int4(j, c0, over ? 0 : cnt, n_e);
  }
}

// 9. packed copy: one wave per chunk of kChunkPieces consecutive pieces of a
// job (the grid covers an upper bound on the chunks; waves past the last exit)
__device__ __forceinline__ PieceArrays piece_arrays(const BJob &J) {
  return piece_arrays(J.s.lay_contig, J.s.piece_off, J.s.piece_len, J.s.piece_src, J.out.len,
                      J.out.base_off);
}

__global__ __launch_bounds__(1024) void kb_copy(BatchDev B) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t gw = blockIdx.x * (blockDim.x / kWave) + wave;
  const int32_t nwv = gridDim.x * (blockDim.x / kWave);
  const int32_t total = ld_const(B.chunk_base, B.n_jobs);
  for (int32_t ch = gw; ch < total; ch += nwv) {
    // a chunk never spans two jobs, so the job is the same for the whole wave
    const CG_CONST uint64_t *pd = (const CG_CONST uint64_t *)(B.chunk_desc + ch);
    const uint64_t d0 = pd[0], d1 = pd[1];
    const int j = (int)(uint32_t)d0, c0 = (int)(uint32_t)(d0 >> 32);
    const int cnt = (int)(uint32_t)d1, n_e = (int)(uint32_t)(d1 >> 32);
    if (cnt <= 0) continue;  // the job's bases overflowed its buffer
    const BJob J = job_at(B.jobs, j);
    copy_chunk(J.g.seq, J.g.seq_words, J.out.bases, piece_arrays(J), c0, cnt, n_e, lane_id());
  }
}

// ---------------------------------------------------------------------------
// Results of a batch in one packed buffer (for a caller that downloads them)
// ---------------------------------------------------------------------------
// Packed record of one job, from its 16-byte aligned start (sizes in
// entries: nc contigs, ne layout entries, tw base words):
//   len u64[nc] | base_off u64[nc] | label, bin, start, n_reads, cflags,
//   layout_off i32[nc] each | layout_vid i32[ne] | bases u32[tw] |
//   layout_rev u8[ne] | zero padding to 16 bytes
constexpr int kCountsBlock = 1024;
constexpr int kPackBlock = 256;

__device__ __forceinline__ int64_t pack_bytes(int64_t nc, int64_t ne, int64_t tw) {
  return (40 * nc + 5 * ne + 4 * tw + 15) & ~(int64_t)15;
}

// out[4j..4j+3] = n_comp, n_e, packed base words, packed offset of job j;
// out[4 n_jobs] = packed bytes of the batch.  One workgroup: a scan over the
// jobs in chunks of its size.
__global__ void __launch_bounds__(kCountsBlock) kb_counts(const BJob *jobs, int n_jobs,
                                                          int64_t *out) {
  __shared__ int64_t part[kCountsBlock / kWave];
  __shared__ int64_t carry;
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int j0 = 0; j0 < n_jobs; j0 += kCountsBlock) {
    const int j = j0 + t;
    int64_t nc = 0, ne = 0, tw = 0, sz = 0;
    if (j < n_jobs) {
      const BJob *J = jobs + j;
      nc = *J->parts.d_n_comp;
      ne = J->local.d_sizes[0];
      tw = (int64_t)*J->out.d_total_words;
      if ((uint64_t)tw > J->out.cap_words) tw = (int64_t)J->out.cap_words;  // not written
      sz = pack_bytes(nc, ne, tw);
    }
    // inclusive scan of sz over the workgroup
    int64_t x = sz;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int64_t y = __shfl_up(x, d, kWave);
      if (lane >= d) x += y;
    }
    if (lane == kWave - 1) part[w] = x;
    __syncthreads();
    int64_t before = carry;
    for (int k = 0; k < w; ++k) before += part[k];
    if (j < n_jobs) {
      out[4 * (int64_t)j + 0] = nc;
      out[4 * (int64_t)j + 1] = ne;
      out[4 * (int64_t)j + 2] = tw;
      out[4 * (int64_t)j + 3] = before + x - sz;
    }
    __syncthreads();
    if (t == kCountsBlock - 1) carry = before + x;
    __syncthreads();
  }
  if (t == 0) out[4 * (int64_t)n_jobs] = carry;
}

// one 4-byte word of the packed results per thread (grid-stride); the job by
// a binary search over the packed offsets, then the segment within it
__global__ void __launch_bounds__(kPackBlock) kb_pack(const BJob *jobs, int n_jobs,
                                                      const int64_t *counts, uint32_t *dst,
                                                      int64_t dst_words) {
  const int64_t total_words = counts[4 * (int64_t)n_jobs] / 4;
  const int64_t lim = total_words < dst_words ? total_words : dst_words;
  for (int64_t wd = (int64_t)blockIdx.x * kPackBlock + threadIdx.x; wd < lim;
       wd += (int64_t)gridDim.x * kPackBlock) {
    const int64_t byte = wd * 4;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (counts[4 * (int64_t)mid + 3] <= byte) lo = mid;
      else hi = mid - 1;
    }
    const int64_t nc = counts[4 * (int64_t)lo], ne = counts[4 * (int64_t)lo + 1];
    const int64_t tw = counts[4 * (int64_t)lo + 2];
    int64_t o = byte - counts[4 * (int64_t)lo + 3];
    const BJob *J = jobs + lo;
    uint32_t v = 0;
    if (o < 16 * nc) {
      const uint32_t *src = (const uint32_t *)(o < 8 * nc ? (const void *)J->out.len
                                                          : (const void *)J->out.base_off);
      v = src[(o < 8 * nc ? o : o - 8 * nc) / 4];
    } else if (o < 40 * nc) {
      const int64_t r = o - 16 * nc, a = r / (4 * nc), i = (r - a * 4 * nc) / 4;
      const uint32_t *src = a == 0 ? (const uint32_t *)J->out.label
                          : a == 1 ? (const uint32_t *)J->out.bin
                          : a == 2 ? (const uint32_t *)J->out.start
                          : a == 3 ? (const uint32_t *)J->out.n_reads
                          : a == 4 ? J->out.cflags
                                   : (const uint32_t *)J->out.layout_off;
      v = src[i];
    } else if ((o -= 40 * nc) < 4 * ne) {
      v = (uint32_t)J->out.layout_vid[o / 4];
    } else if ((o -= 4 * ne) < 4 * tw) {
      v = J->out.bases[o / 4];
    } else {
      o -= 4 * tw;
      for (int k = 0; k < 4; ++k)
        if (o + k < ne) v |= (uint32_t)J->out.layout_rev[o + k] << (8 * k);
    }
    dst[wd] = v;
  }
}

}  // namespace cg

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
using namespace cg;

struct cg_batch {
  cg_ctx *ctx;
  int32_t n_jobs, n_vtiles;
  int32_t n_internal;  // jobs the batched launches run (the others are external)
  const MaskTile *mtiles;  // [dev.n_mtiles] tiles of kb_mask_tiles
  bool any_bases;   // a job partitioned by bases weights
  int64_t chunk_slots;  // upper bound on the copy chunks of the batch
  // workgroups of each per-component pass that fit on the device at once:
  // their grids stay within it, so every workgroup of the snake order runs
  // from the start (a workgroup that waits for a free slot starts its whole
  // share late)
  int res_iw_tiny, res_iw_small, res_iw, res_walk;
  // jobs too large for one workgroup's components pass: they run through the
  // single-graph kernels (grid-wide) ahead of the batched launches
  std::vector<cg_job> ext_jobs;
  std::vector<Scratch> ext_s;
  cg_batch_params prm;
  BatchDev dev;
  char *mem;
  size_t mem_bytes;
  hipGraph_t graph;
  hipGraphExec_t exec;
  // host copies of the tables of the current plan (kept until the next plan:
  // a plan's uploads may still read them)
  std::vector<BJob> h_jobs;
  std::vector<int32_t> h_tiles, h_order;
  std::vector<MaskTile> h_mtiles;
};

// sizes and parameters of a job (all that its share of the batch memory
// depends on)
static int check_job_sizes(const cg_job &J, int i) {
  if (J.g.n < 0 || J.g.n >= (1 << 30) || J.g.m < 0)
    return set_error(CG_EINVAL, "job %d: n=%d m=%d", i, J.g.n, J.g.m);
  if (J.P < 1 || J.P > 65536) return set_error(CG_EINVAL, "job %d: P=%d outside [1, 65536]", i, J.P);
  if (J.weight != CG_WEIGHT_READS && J.weight != CG_WEIGHT_BASES)
    return set_error(CG_EINVAL, "job %d: weight=%d", i, J.weight);
  return CG_OK;
}

static int check_job(const cg_job &J, int i) {
  const cg_graph &g = J.g;
  int rc = check_job_sizes(J, i);
  if (rc) return rc;
  if (!g.row_ptr || (g.m > 0 && (!g.col || !g.ovl || !g.strand)) ||
      (g.n > 0 && (!g.read_len || !g.read_off || !g.seq)) || ((g.pre == nullptr) != (g.post == nullptr)))
    return set_error(CG_EINVAL, "job %d: bad graph", i);
  const cg_parts &p = J.parts;
  const cg_local &l = J.local;
  const cg_contigs &c = J.contigs;
  if (!J.flags || !J.d_counts || !J.label || !p.comp_label || !p.comp_size || !p.comp_kind ||
      !p.comp_bin || !p.comp_rank || !p.comp_start || !p.bin_load || !p.label_comp ||
      !p.d_n_comp || !l.perm || !l.bin_vptr || !l.loc_row_ptr || !l.loc_col || !l.loc_eid ||
      !l.d_sizes || !c.label || !c.bin || !c.start || !c.n_reads || !c.len || !c.base_off ||
      !c.cflags || !c.layout_off || !c.layout_vid || !c.layout_rev || !c.d_total_words ||
      (c.cap_words > 0 && !c.bases))
    return set_error(CG_EINVAL, "job %d: a buffer is NULL", i);
  // the mask and components pass moves reads with 16-byte accesses
  if (((uintptr_t)g.row_ptr & 15) || ((uintptr_t)J.label & 15) || ((uintptr_t)p.label_comp & 15) ||
      ((uintptr_t)J.flags & 15))
    return set_error(CG_EINVAL,
                     "job %d: row_ptr, flags, label and label_comp must be 16-byte aligned", i);
  return CG_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Where every table of a batch lives in its device memory, for one set of
// jobs (sizes only; plan_fill writes the tables).
struct Plan {
  int32_t n_jobs = 0, nv = 0, n_mt = 0, n_internal = 0;
  int64_t sum_chunks = 0;
  bool any_bases = false;
  size_t o_jobs, o_tiles, o_cbase, o_pbase, o_hbase, o_jcnt, o_cjob, o_wq, o_wqh, o_wqc, o_wqm,
      o_hjob, o_counters, o_order, o_mtiles, o_mtcnt, o_ccp, total = 0;
  std::vector<size_t> job_off;
};

static int check_params(cg_ctx *ctx, const cg_batch_params *params, cg_batch_params *out) {
  cg_batch_params prm = params ? *params : cg_batch_params{0, 0, 0};
  if (prm.vertex_tile == 0) prm.vertex_tile = 256;
  if (prm.vertex_tile != 256 && prm.vertex_tile != 512 && prm.vertex_tile != 1024)
    return set_error(CG_EINVAL, "vertex_tile must be 256, 512 or 1024");
  if (prm.copy_block == 0) prm.copy_block = 256;
  if (prm.copy_block < 64 || prm.copy_block > 1024 || prm.copy_block % 64)
    return set_error(CG_EINVAL, "copy_block must be a multiple of 64 in [64, 1024]");
  if (prm.persist_blocks == 0) {
    hipDeviceProp_t prop;
    int rc = hip_check(hipGetDeviceProperties(&prop, ctx->device), "hipGetDeviceProperties");
    if (rc) return rc;
    prm.persist_blocks = 4 * prop.multiProcessorCount;
  }
  if (prm.persist_blocks < 1) return set_error(CG_EINVAL, "persist_blocks must be positive");
  *out = prm;
  return CG_OK;
}

// sizes and offsets of a plan for these jobs (checks every job: all of it,
// or with sizes_only its sizes and parameters)
static int plan_sizes(int32_t n_jobs, const cg_job *jobs, int vertex_tile, Plan *P,
                      bool sizes_only = false) {
  if (!jobs || n_jobs < 1) return set_error(CG_EINVAL, "a batch needs at least one job");
  int64_t total_n = 0;
  for (int i = 0; i < n_jobs; ++i) {
    int rc = sizes_only ? check_job_sizes(jobs[i], i) : check_job(jobs[i], i);
    if (rc) return rc;
    total_n += jobs[i].g.n + 1;
  }
  if (total_n >= (1ll << 31)) return set_error(CG_EUNSUPPORTED, "batch holds 2^31 or more reads");
  const int T = vertex_tile;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t here = at;
    at += align256(bytes);
    return here;
  };
  P->n_jobs = n_jobs;
  P->o_jobs = take(sizeof(BJob) * n_jobs);
  P->nv = 0;
  for (int i = 0; i < n_jobs; ++i) P->nv += (int32_t)((jobs[i].g.n + 1 + T - 1) / T);
  P->o_tiles = take(sizeof(int32_t) * P->nv);
  P->o_cbase = take(sizeof(int32_t) * (n_jobs + 1));
  P->o_pbase = take(sizeof(int32_t) * (n_jobs + 1));
  P->o_hbase = take(sizeof(int32_t) * (n_jobs + 1));
  P->o_ccp = take(sizeof(int32_t) * n_jobs);
  P->o_jcnt = take(sizeof(int2) * n_jobs);
  int64_t sum_n = 0;
  P->sum_chunks = 0;
  P->any_bases = false;
  int64_t max_n = 0;
  for (int i = 0; i < n_jobs; ++i) {
    sum_n += jobs[i].g.n;
    max_n = jobs[i].g.n > max_n ? jobs[i].g.n : max_n;
    P->sum_chunks += (jobs[i].g.n + kChunkPieces - 1) / kChunkPieces;
    P->any_bases |= jobs[i].weight == CG_WEIGHT_BASES;
  }
  // the tail chunks: the jobs in the last sixteenth of the pieces hold at
  // most a sixteenth of all reads plus one job's, in chunks of
  // kTailChunkPieces (one partial chunk per job)
  P->sum_chunks += (sum_n / 16 + max_n) / kTailChunkPieces + n_jobs + 1;
  P->o_cjob = take(sizeof(int32_t) * (size_t)(sum_n > 0 ? sum_n : 1));
  P->o_wq = take(sizeof(WqE) * (size_t)(sum_n > 0 ? sum_n : 1));
  P->o_wqh = take(sizeof(int32_t) * kWqBuckets);
  P->o_wqc = take(sizeof(int32_t) * kWqBuckets);
  P->o_wqm = take(sizeof(int32_t) * 8);
  P->o_hjob = take(sizeof(int4) * (size_t)(P->sum_chunks > 0 ? P->sum_chunks : 1));
  P->o_counters = take(sizeof(unsigned int) * 8);
  P->o_order = take(sizeof(int32_t) * n_jobs);
  P->job_off.resize(n_jobs);
  P->n_internal = P->n_mt = 0;
  for (int i = 0; i < n_jobs; ++i) {
    // the components pass holds a job's reads as LDS bitmaps and its reads
    // of degree 1-2 (at most its entries) in LDS; larger jobs go through the
    // single-graph kernels
    const bool ext = jobs[i].g.n > kMcReadCap || jobs[i].g.m > kExternalEntries;
    P->n_internal += ext ? 0 : 1;
    P->n_mt += ext ? 0 : (jobs[i].g.n + kMaskTile - 1) / kMaskTile;
    P->job_off[i] = take(layout(jobs[i].g.n, jobs[i].g.m, jobs[i].P).total);
  }
  P->o_mtiles = take(sizeof(MaskTile) * (P->n_mt > 0 ? P->n_mt : 1));
  P->o_mtcnt = take(sizeof(int2) * (P->n_mt > 0 ? P->n_mt : 1));
  P->total = at;
  return CG_OK;
}

// the plan's tables for the batch memory at b->mem, in b's host copies, and
// b's fields and device pointers; the tables still have to be uploaded
static void plan_fill(cg_batch *b, const Plan &P, const cg_job *jobs) {
  const int n_jobs = P.n_jobs;
  const int T = b->prm.vertex_tile;
  char *mem = b->mem;
  b->h_jobs.assign(n_jobs, BJob{});
  b->h_tiles.clear();
  b->h_mtiles.clear();
  b->h_order.resize(n_jobs);
  b->ext_jobs.clear();
  b->ext_s.clear();
  int2 *d_mtcnt = (int2 *)(mem + P.o_mtcnt);
  int32_t nv = 0, n_mt = 0;
  for (int i = 0; i < n_jobs; ++i) {
    const cg_job &J = jobs[i];
    BJob &h = b->h_jobs[i];
    h.g = J.g;
    h.P = J.P;
    h.min_reads = J.min_reads;
    h.weight = J.weight;
    h.flags = J.flags;
    h.counts = J.d_counts;
    h.label = J.label;
    h.parts = J.parts;
    h.local = J.local;
    h.out = J.contigs;
    const int32_t cnt = (int32_t)((J.g.n + 1 + T - 1) / T);
    h.vt_first = nv;
    h.vt_count = cnt;
    for (int32_t t = 0; t < cnt; ++t) b->h_tiles.push_back(i);
    nv += cnt;
    h.external = (J.g.n > kMcReadCap || J.g.m > kExternalEntries) ? 1 : 0;
    // carve this job's scratch slice the way a context carves its scratch
    cg_ctx view{};
    view.scratch = mem + P.job_off[i];
    view.scratch_bytes = layout(J.g.n, J.g.m, J.P).total;
    carve(&view, J.g.n, J.g.m, J.P, &h.s);
    h.mt_first = n_mt;
    h.mt_count = h.external ? 0 : (J.g.n + kMaskTile - 1) / kMaskTile;
    // the mask tiles: the job's lists live in its walk scratch, its bitmaps
    // in its fill scratch (both reused by later steps)
    for (int32_t v0 = 0; !h.external && v0 < J.g.n; v0 += kMaskTile)
      b->h_mtiles.push_back(MaskTile{J.g.row_ptr, J.g.col, (int4 *)h.s.walk,
                                     (uint32_t *)h.s.fill, d_mtcnt + n_mt++, J.flags, J.label,
                                     J.parts.label_comp, J.g.n, v0, (J.g.n + 31) / 32, 0});
    if (h.external) {
      b->ext_jobs.push_back(J);
      b->ext_s.push_back(h.s);
    }
  }
  for (int i = 0; i < n_jobs; ++i) b->h_order[i] = i;
  std::stable_sort(b->h_order.begin(), b->h_order.end(),
                   [&](int a, int c) { return jobs[a].g.n > jobs[c].g.n; });
  b->n_jobs = n_jobs;
  b->n_vtiles = nv;
  b->chunk_slots = P.sum_chunks;
  b->n_internal = P.n_internal;
  b->any_bases = P.any_bases;
  b->mtiles = (const MaskTile *)(mem + P.o_mtiles);
  BatchDev &d = b->dev;
  d.jobs = (BJob *)(mem + P.o_jobs);
  d.tile_job = (int32_t *)(mem + P.o_tiles);
  d.comp_base = (int32_t *)(mem + P.o_cbase);
  d.piece_base = (int32_t *)(mem + P.o_pbase);
  d.chunk_base = (int32_t *)(mem + P.o_hbase);
  d.chunk_cp = (int32_t *)(mem + P.o_ccp);
  d.job_cnt = (int2 *)(mem + P.o_jcnt);
  d.wq = (WqE *)(mem + P.o_wq);
  d.wq_hist = (int32_t *)(mem + P.o_wqh);
  d.wq_cur = (int32_t *)(mem + P.o_wqc);
  d.wq_meta = (int32_t *)(mem + P.o_wqm);
  d.comp_job = (int32_t *)(mem + P.o_cjob);
  d.chunk_desc = (int4 *)(mem + P.o_hjob);
  d.counters = (unsigned int *)(mem + P.o_counters);
  d.job_order = (const int32_t *)(mem + P.o_order);
  d.mt_cnt = d_mtcnt;
  d.n_mtiles = n_mt;
  d.fixed = b->ctx->fixed;
  d.n_jobs = n_jobs;
  d.n_vtiles = nv;
}

// enqueue the plan's uploads on st (tables from b's host copies); the
// launch counters are cleared by a small kernel (no memset node, so the
// sequence can sit in a captured graph)
__global__ void kb_clear_counters(unsigned int *c) {
  if (threadIdx.x < 8) c[threadIdx.x] = 0;
}

// the look-back status words of a job that runs through the single-graph
// kernels start at zero (its slice of the batch memory may hold anything
// from an earlier plan)
__global__ void kb_clear_status(unsigned long long *p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

static int plan_upload(cg_batch *b, const Plan &P, hipStream_t st) {
  char *mem = b->mem;
  int rc = hip_check(hipMemcpyAsync(mem + P.o_jobs, b->h_jobs.data(), sizeof(BJob) * P.n_jobs,
                                    hipMemcpyHostToDevice, st), "hipMemcpyAsync(jobs)");
  if (!rc && P.nv > 0)
    rc = hip_check(hipMemcpyAsync(mem + P.o_tiles, b->h_tiles.data(), sizeof(int32_t) * P.nv,
                                  hipMemcpyHostToDevice, st), "hipMemcpyAsync(tiles)");
  if (!rc)
    rc = hip_check(hipMemcpyAsync(mem + P.o_order, b->h_order.data(), sizeof(int32_t) * P.n_jobs,
                                  hipMemcpyHostToDevice, st), "hipMemcpyAsync(job order)");
  if (!rc && P.n_mt > 0)
    rc = hip_check(hipMemcpyAsync(mem + P.o_mtiles, b->h_mtiles.data(),
                                  sizeof(MaskTile) * P.n_mt, hipMemcpyHostToDevice, st),
                   "hipMemcpyAsync(mask tiles)");
  if (!rc) {
    hipLaunchKernelGGL(kb_clear_counters, dim3(1), dim3(64), 0, st, b->dev.counters);
    rc = hip_check(hipGetLastError(), "kb_clear_counters");
  }
  for (size_t e = 0; !rc && e < b->ext_jobs.size(); ++e) {
    const int words = scan_blocks((int64_t)(b->ext_jobs[e].g.n > 0 ? b->ext_jobs[e].g.n : 1) + 1) + 1;
    hipLaunchKernelGGL(kb_clear_status, dim3((words + 255) / 256), dim3(256), 0, st,
                       b->ext_s[e].scan_status, words);
    rc = hip_check(hipGetLastError(), "kb_clear_status");
  }
  return rc;
}

static int batch_alloc(cg_ctx *ctx, const cg_batch_params &prm, size_t bytes, cg_batch **out) {
  cg_batch *b = new (std::nothrow) cg_batch();
  if (!b) return set_error(CG_EINVAL, "out of host memory");
  b->ctx = ctx;
  b->prm = prm;
  b->n_jobs = b->n_vtiles = b->n_internal = 0;
  b->any_bases = false;
  b->chunk_slots = 0;
  b->mtiles = nullptr;
  b->graph = nullptr;
  b->exec = nullptr;
  b->mem = nullptr;
  b->mem_bytes = bytes > 0 ? bytes : 256;
  {
    int dev = 0, cus = 0, k0 = 0, k1 = 0, k3 = 0, k4 = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&k0, kb_induce_walk_tiny, kWalkSmallBlock,
                                                     0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&k1, kb_induce_walk_small, kWalkSmallBlock,
                                                     0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&k3, kb_induce_walk, kWalkBlock, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&k4, kb_walk, kWalkBlock, 0) != hipSuccess) {
      delete b;
      return set_error(CG_EHIP, "occupancy query failed");
    }
    b->res_iw_tiny = k0 * cus;
    b->res_iw_small = k1 * cus;
    b->res_iw = k3 * cus;
    b->res_walk = k4 * cus;
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  int rc = hip_check(hipMalloc((void **)&b->mem, b->mem_bytes), "hipMalloc(batch)");
  if (!rc) rc = hip_check(hipMemset(b->mem, 0, b->mem_bytes), "hipMemset(batch)");
  (void)hipSetDevice(prev);
  if (rc) {
    if (b->mem) (void)hipFree(b->mem);
    delete b;
    return rc;
  }
  *out = b;
  return CG_OK;
}

extern "C" {

int cg_batch_bytes(int32_t n_jobs, const cg_job *jobs, const cg_batch_params *params,
                   uint64_t *bytes) {
  if (!bytes) return set_error(CG_EINVAL, "bytes is NULL");
  const int T = params && params->vertex_tile ? params->vertex_tile : 256;
  if (T != 256 && T != 512 && T != 1024)
    return set_error(CG_EINVAL, "vertex_tile must be 256, 512 or 1024");
  Plan P;
  int rc = plan_sizes(n_jobs, jobs, T, &P, true);
  if (rc) return rc;
  *bytes = (uint64_t)P.total;
  return CG_OK;
}

int cg_batch_create(cg_ctx *ctx, int32_t n_jobs, const cg_job *jobs,
                    const cg_batch_params *params, cg_batch **out) {
  if (!ctx || !jobs || !out || n_jobs < 1) return set_error(CG_EINVAL, "bad batch arguments");
  *out = nullptr;
  cg_batch_params prm;
  int rc = check_params(ctx, params, &prm);
  if (rc) return rc;
  Plan P;
  if ((rc = plan_sizes(n_jobs, jobs, prm.vertex_tile, &P))) return rc;
  cg_batch *b = nullptr;
  if ((rc = batch_alloc(ctx, prm, P.total, &b))) return rc;
  plan_fill(b, P, jobs);
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  rc = plan_upload(b, P, nullptr);
  if (!rc) rc = hip_check(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
  (void)hipSetDevice(prev);
  if (rc) {
    (void)hipFree(b->mem);
    delete b;
    return rc;
  }
  *out = b;
  return CG_OK;
}

int cg_batch_create_empty(cg_ctx *ctx, uint64_t bytes, const cg_batch_params *params,
                          cg_batch **out) {
  if (!ctx || !out) return set_error(CG_EINVAL, "bad batch arguments");
  *out = nullptr;
  cg_batch_params prm;
  int rc = check_params(ctx, params, &prm);
  if (rc) return rc;
  return batch_alloc(ctx, prm, (size_t)bytes, out);
}

int cg_batch_plan(cg_batch *b, int32_t n_jobs, const cg_job *jobs, void *stream) {
  if (!b) return set_error(CG_EINVAL, "batch is NULL");
  Plan P;
  int rc = plan_sizes(n_jobs, jobs, b->prm.vertex_tile, &P);
  if (rc) return rc;
  if (P.total > b->mem_bytes)
    return set_error(CG_ECAPACITY, "the jobs need %zu bytes of batch memory, the batch has %zu",
                     P.total, b->mem_bytes);
  // a captured graph holds the previous plan's launch shapes
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  plan_fill(b, P, jobs);
  return plan_upload(b, P, (hipStream_t)stream);
}

int cg_batch_run(cg_batch *b, void *stream) {
  if (!b) return set_error(CG_EINVAL, "batch is NULL");
  if (b->n_jobs < 1) return set_error(CG_EINVAL, "batch has no jobs (cg_batch_plan)");
  hipStream_t st = (hipStream_t)stream;
  cg_ctx *ctx = b->ctx;
  const BatchDev &B = b->dev;
  const int T = b->prm.vertex_tile;
  const int PB = b->prm.persist_blocks;
  for (size_t e = 0; e < b->ext_jobs.size(); ++e) {
    const cg_job &J = b->ext_jobs[e];
    const Scratch &s = b->ext_s[e];
    int rc = launch_mask(ctx, J.g, J.flags, J.d_counts, st);
    if (!rc) rc = launch_components(ctx, J.g, J.flags, J.label, st);
    if (!rc)
      rc = launch_partition(ctx, J.g, s, J.flags, J.label, J.P, J.min_reads, J.weight, J.parts, st);
    if (!rc) rc = launch_induce(ctx, J.g, s, J.flags, J.label, J.parts, J.P, J.local, st);
    if (!rc) rc = launch_assemble(ctx, J.g, s, J.parts, J.local, J.P, J.contigs, st);
    if (rc) return rc;
  }
  if (b->n_internal == 0) return hip_check(hipGetLastError(), "cg_batch_run");
  {
    const PhaseRange range("cg_batch: BranchRemoval + ConnectedComponent");
    if (B.n_mtiles > 0)
      CG_LAUNCH(ctx, kb_mask_tiles, dim3(B.n_mtiles), dim3(kMaskThreads), st, b->mtiles);
    CG_LAUNCH(ctx, kb_mask_cc, dim3(b->n_jobs), dim3(kMcBlock), st, B);
  }
  const PhaseRange range_p("cg_batch: GreedyPartitioning, InducedSubgraph, LocalAssembly");
  if (b->any_bases) {
    if (T == 256) CG_LAUNCH(ctx, kb_weight<256>, dim3(b->n_vtiles), dim3(256), st, B);
    else if (T == 512) CG_LAUNCH(ctx, kb_weight<512>, dim3(b->n_vtiles), dim3(512), st, B);
    else CG_LAUNCH(ctx, kb_weight<1024>, dim3(b->n_vtiles), dim3(1024), st, B);
  }
  CG_LAUNCH(ctx, kb_lpt, dim3(b->n_jobs), dim3(kBatchLptBlock), st, B);
  CG_LAUNCH(ctx, kb_tables, dim3(256), dim3(kTablesBlock), st, B);
  CG_LAUNCH(ctx, kb_wq_place, dim3(128), dim3(kWqBlock), st, B);
  auto capped = [](int want, int fit) { return dim3((unsigned)(fit > 0 && fit < want ? fit : want)); };
  // components above kIwCap reads in two passes (the induce step with the
  // next ones, the walk after the last pass that reads the tile lists, since
  // its arrays take their memory), the others in one
  CG_LAUNCH(ctx, kb_induce_walk, capped(PB, b->res_iw), dim3(kWalkBlock), st, B);
  CG_LAUNCH(ctx, kb_induce_walk_small, capped(4 * PB, b->res_iw_small), dim3(kWalkSmallBlock), st,
            B);
  CG_LAUNCH(ctx, kb_induce_walk_tiny, capped(8 * PB, b->res_iw_tiny), dim3(kWalkSmallBlock), st,
            B);
  CG_LAUNCH(ctx, kb_walk, capped(PB, b->res_walk), dim3(kWalkBlock), st, B);
  CG_LAUNCH(ctx, kb_offsets, dim3(b->n_jobs), dim3(kScanBlock), st, B);
  // one wave per copy chunk slot: the hardware hands chunks to waves as
  // slots free up (a persistent grid with a fixed share per wave left a
  // tail of unevenly loaded waves); slots past the batch's chunks exit
  const int64_t wpb = b->prm.copy_block / kWave;
  const int64_t cgrid = (b->chunk_slots + wpb - 1) / wpb;
  CG_LAUNCH(ctx, kb_copy, dim3((unsigned)(cgrid > 0 ? cgrid : 1)), dim3(b->prm.copy_block), st, B);
  return hip_check(hipGetLastError(), "cg_batch_run");
}

int cg_batch_counts(cg_batch *b, int64_t *d_counts, void *stream) {
  if (!b || !d_counts) return set_error(CG_EINVAL, "bad arguments");
  if (b->n_jobs < 1) return set_error(CG_EINVAL, "batch has no jobs (cg_batch_plan)");
  CG_LAUNCH(b->ctx, kb_counts, dim3(1), dim3(kCountsBlock), (hipStream_t)stream, b->dev.jobs,
            b->n_jobs, d_counts);
  return hip_check(hipGetLastError(), "cg_batch_counts");
}

int cg_batch_pack(cg_batch *b, const int64_t *d_counts, void *d_dst, uint64_t dst_bytes,
                  void *stream) {
  if (!b || !d_counts || (dst_bytes > 0 && !d_dst)) return set_error(CG_EINVAL, "bad arguments");
  if (b->n_jobs < 1) return set_error(CG_EINVAL, "batch has no jobs (cg_batch_plan)");
  if ((uintptr_t)d_dst & 15) return set_error(CG_EINVAL, "d_dst must be 16-byte aligned");
  if (dst_bytes < 4) return CG_OK;
  int dev = 0, cus = 0;
  int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (!rc) rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
                          "hipDeviceGetAttribute");
  if (rc) return rc;
  const int64_t words = (int64_t)(dst_bytes / 4);
  int64_t grid = (words + kPackBlock - 1) / kPackBlock;
  if (grid > 8 * (int64_t)cus) grid = 8 * (int64_t)cus;
  CG_LAUNCH(b->ctx, kb_pack, dim3((unsigned)grid), dim3(kPackBlock), (hipStream_t)stream,
            b->dev.jobs, b->n_jobs, d_counts, (uint32_t *)d_dst, words);
  return hip_check(hipGetLastError(), "cg_batch_pack");
}

int cg_batch_capture(cg_batch *b, void *stream) {
  if (!b || !stream) return set_error(CG_EINVAL, "capture needs a batch and a non-default stream");
  hipStream_t st = (hipStream_t)stream;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  // kernels only: per-kernel event timing stays off while capturing
  ProfEntry *saved = b->ctx->prof;
  b->ctx->prof = nullptr;
  int rc = hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal),
                     "hipStreamBeginCapture");
  if (!rc) {
    int rr = cg_batch_run(b, stream);
    rc = hip_check(hipStreamEndCapture(st, &b->graph), "hipStreamEndCapture");
    if (!rc) rc = rr;
  }
  b->ctx->prof = saved;
  if (!rc) rc = hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0),
                          "hipGraphInstantiate");
  return rc;
}

int cg_batch_launch(cg_batch *b, void *stream) {
  if (!b || !b->exec) return set_error(CG_EINVAL, "batch has no captured graph");
  return hip_check(hipGraphLaunch(b->exec, (hipStream_t)stream), "hipGraphLaunch");
}

int cg_batch_destroy(cg_batch *b) {
  if (!b) return CG_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  int rc = CG_OK;
  if (b->mem) rc = hip_check(hipFree(b->mem), "hipFree(batch)");
  delete b;
  return rc;
}

}  // extern "C"
