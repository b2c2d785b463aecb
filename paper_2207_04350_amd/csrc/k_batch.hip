// Batched form: the five steps of Algorithm 2 for many independent string
// graphs ("jobs") with one launch per phase for the whole batch.
//
//  vertex passes   each job is cut into tiles of T vertices; a launch covers
//                  the tiles of every job (tile -> job table)
//  compaction      reduce-then-scan per job: tiles count, then each tile adds
//                  up the counts of the tiles before it in its job
//  component and   persistent grids over the batch-wide item ranges
//  piece passes    (components, pieces) whose per-job bases the last LPT
//                  workgroup computes on the device; the per-component passes
//                  take a work queue of every component of the batch in
//                  decreasing read count
//
// Every counter a launch uses is reset by the launch itself, and the
// union-find forest is reset by bumping its tag, so the launches (twelve, or
// more when one-read components are eligible or weights are bases) can be
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
  uint64_t *forest;            // [n] tagged union-find forest (batch-owned, never reused)
  int4 *conn_list;             // [n] reads of degree 1-2, each mask tile's reads packed in id
                               // order at the start of its slice: (id, columns or -1, degree)
                               // from the mask pass, then (id, s0, s1, kept bits) from the
                               // neighbour pass, s_k the list slot of neighbour k when its
                               // entry is kept and its id is smaller, else -1
  int32_t *conn_map;           // [n] slot of a listed read in conn_list
  int32_t vt_first, vt_count;  // the job's vertex tiles (covering 0..n)
  int32_t mt_first, mt_count;  // the job's mask tiles
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

// One tile of the mask pass: kMaskTile consecutive reads of one job.
struct MaskTile {
  const int32_t *row_ptr;
  const int32_t *col;
  uint8_t *flags;
  int32_t *label;
  int32_t *label_comp;
  int4 *conn_list;
  int32_t *conn_map;
  int2 *tile_cnt;   // (listed reads, branch reads) of this tile
  int32_t n, v0;
  int32_t lc_init;  // first value of label_comp: -1, or 4 (one-read count) when
                    // one-read components can be eligible
  int32_t pad_;
};
static_assert(sizeof(MaskTile) % 8 == 0, "tile descriptors are copied in 8-byte words");
constexpr int kMaskThreads = 256;
constexpr int kMaskGroups = 2;  // groups of 4 consecutive reads per thread
constexpr int kMaskTile = 4 * kMaskThreads * kMaskGroups;

struct BatchDev {
  BJob *jobs;                       // [n_jobs]
  int32_t *tile_job;                // [n_vtiles]
  int32_t *tile_cnt;                // [n_vtiles] eligible roots per tile
  int32_t *comp_base;               // [n_jobs + 1] first component item of each job
  int32_t *piece_base;              // [n_jobs + 1] first piece item of each job
  int32_t *chunk_base;              // [n_jobs + 1] first 64-piece copy chunk of each job
  int2 *job_cnt;                    // [n_jobs] (components, component reads) of each job
  // work queue of the per-component passes: every component of the batch as
  // (job, component, reads, first local number), in decreasing read count
  int4 *wq;                         // [upper bound on the batch's components]
  int32_t *wq_hist;                 // [kWqBuckets] components per read count (capped)
  int32_t *wq_cur;                  // [kWqBuckets] placement cursors
  int32_t *wq_meta;                 // [8] 0: components, 1: those above kWalkSmallCap
                                    // reads, 2: above kIndSmallCap
  int32_t *comp_job;                // [sum n] job of each batch-wide component
  int32_t *chunk_job;               // [sum of ceil(n / kChunkPieces)] job of each copy chunk
  unsigned int *counters;           // [8] 2: LPT ticket, 3: runs so far (forest tag - 1)
  int2 *mt_cnt;                     // [n_mtiles] (listed reads, branch reads) of each mask tile
  const int32_t *job_order;         // [n_jobs] jobs by decreasing read count
  const MaskTile *mtiles;           // [n_mtiles]
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
// 1. mask (eight reads per thread as two 16-byte row_ptr sweeps): branch
// flags, labels and label_comp initialised, and every read of degree 1-2
// listed with its columns, packed per tile in id order by a block scan.
// Whether an entry is kept needs the other end's branch bit, which the
// job's components workgroup reads next, from the job's flags.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t forest_tag(const BatchDev &B) { return B.counters[3] + 1u; }

__global__ __launch_bounds__(kMaskThreads) void kb_mask_list(const MaskTile *__restrict__ tiles) {
  __shared__ int64_t sh[kMaskThreads / kWave + 1];
  const MaskTile D = tiles[blockIdx.x];
  const int32_t n = D.n;
  const int lane = lane_id();
  int32_t v0[kMaskGroups];
  int4 a[kMaskGroups];
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g) {
    v0[g] = D.v0 + g * 4 * kMaskThreads + 4 * (int32_t)threadIdx.x;
    a[g] = make_int4(0, 0, 0, 0);
    if (v0[g] + 3 <= n) {
      a[g] = *(const int4 *)(D.row_ptr + v0[g]);
    } else if (v0[g] <= n) {
      a[g].x = D.row_ptr[v0[g]];
      if (v0[g] + 1 <= n) a[g].y = D.row_ptr[v0[g] + 1];
      if (v0[g] + 2 <= n) a[g].z = D.row_ptr[v0[g] + 2];
    }
  }
  int32_t e4[kMaskGroups];
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g) {
    e4[g] = __shfl_down(a[g].x, 1);
    if (lane == kWave - 1 && v0[g] + 4 <= n) e4[g] = D.row_ptr[v0[g] + 4];
  }
  constexpr int R = 4 * kMaskGroups;
  int32_t dg[R], bb[R];
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g) {
    const int32_t rp[5] = {a[g].x, a[g].y, a[g].z, a[g].w, e4[g]};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dg[4 * g + i] = v0[g] + i < n ? rp[i + 1] - rp[i] : 0;
      bb[4 * g + i] = rp[i];
    }
  }
  int32_t u0[R], u1[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    u0[k] = (dg[k] == 1 || dg[k] == 2) ? D.col[bb[k]] : -1;
    u1[k] = dg[k] == 2 ? D.col[bb[k] + 1] : -1;
  }
  // listed reads packed in id order: group 0 of every thread precedes group
  // 1, so one scan of (listed, branch) counts of both groups, 16-bit fields
  // (a tile holds fewer than 2^16 reads), gives every position.  The scan
  // comes before any store: its barriers would wait for them.
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
  int32_t pos[kMaskGroups] = {D.v0 + (int32_t)(ex & 0xFFFF), D.v0 + listed0 + (int32_t)((ex >> 32) & 0xFFFF)};
#pragma unroll
  for (int g = 0; g < kMaskGroups; ++g) {
    uint32_t fw = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) fw |= (dg[4 * g + i] >= 3 ? 1u : 0u) << (8 * i);
    const int32_t v = v0[g];
    if (v + 3 < n) {
      *(uint32_t *)(D.flags + v) = fw;
      *(int4 *)(D.label + v) = make_int4(v, v + 1, v + 2, v + 3);
      *(int4 *)(D.label_comp + v) = make_int4(D.lc_init, D.lc_init, D.lc_init, D.lc_init);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (v + i < n) {
          D.flags[v + i] = (uint8_t)(fw >> (8 * i));
          D.label[v + i] = v + i;
          D.label_comp[v + i] = D.lc_init;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * g + i;
      if (dg[k] == 1 || dg[k] == 2) {
        D.conn_list[pos[g]] = make_int4(v0[g] + i, u0[k], u1[k], dg[k]);
        D.conn_map[v0[g] + i] = pos[g];
        ++pos[g];
      }
    }
  }
  if (threadIdx.x == 0)
    *D.tile_cnt = make_int2(listed0 + (int32_t)((tot >> 32) & 0xFFFF),
                            (int32_t)((tot >> 16) & 0xFFFF) + (int32_t)((tot >> 48) & 0xFFFF));
}

// 1b. the neighbour lookups of every listed read, spread over the whole chip
// (done inside the components pass they would fall on one CU per job): kept
// bits from the neighbours' branch bits, and the list slots of the kept
// neighbours with smaller ids, written back into the read's list entry
constexpr int kPrepChunks = kMaskTile / kMaskThreads;
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kMaskThreads) void kb_cc_prep(const MaskTile *__restrict__ tiles) {
  // the tile descriptor through the constant address space (scalar loads),
  // its arrays as global memory
  MaskTile D;
  {
    const CG_CONST uint64_t *p = (const CG_CONST uint64_t *)(tiles + blockIdx.x);
    uint64_t *q = reinterpret_cast<uint64_t *>(&D);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(MaskTile) / 8); ++k) q[k] = p[k];
  }
  const int32_t c = ((const CG_GLOBAL int2 *)D.tile_cnt)->x;
  if (c == 0) return;
  CG_GLOBAL i32x4 *list = (CG_GLOBAL i32x4 *)D.conn_list + D.v0;
  const CG_GLOBAL uint8_t *flags = (const CG_GLOBAL uint8_t *)D.flags;
  const CG_GLOBAL int32_t *map = (const CG_GLOBAL int32_t *)D.conn_map;
  // all loads of the thread's entries in flight before any is used; slots at
  // or past c read slot 0 and are then treated as empty (a listed read's
  // job has at least one read, so index 0 is in bounds)
  i32x4 e[kPrepChunks];
#pragma unroll
  for (int k = 0; k < kPrepChunks; ++k) {
    const int32_t i = k * kMaskThreads + (int32_t)threadIdx.x;
    e[k] = list[i < c ? i : 0];
  }
  uint32_t b0[kPrepChunks], b1[kPrepChunks];
  int32_t m0[kPrepChunks], m1[kPrepChunks];
#pragma unroll
  for (int k = 0; k < kPrepChunks; ++k) {
    const int32_t i = k * kMaskThreads + (int32_t)threadIdx.x;
    if (i >= c) e[k] = i32x4{-1, -1, -1, 0};
    const int32_t u0 = e[k].y >= 0 ? e[k].y : 0, u1 = e[k].z >= 0 ? e[k].z : 0;
    b0[k] = flags[u0];
    b1[k] = flags[u1];
    m0[k] = map[u0];
    m1[k] = map[u1];
  }
#pragma unroll
  for (int k = 0; k < kPrepChunks; ++k) {
    const int32_t i = k * kMaskThreads + (int32_t)threadIdx.x;
    if (i >= c) continue;
    const bool k0 = e[k].y >= 0 && !(b0[k] & 1), k1 = e[k].z >= 0 && !(b1[k] & 1);
    list[i] = i32x4{e[k].x, k0 && e[k].y < e[k].x ? m0[k] : -1, k1 && e[k].z < e[k].x ? m1[k] : -1,
                    (k0 ? 2 : 0) | (k1 ? 4 : 0)};
  }
}

// 2. components of each job in one workgroup, from its listed reads: kept
// bits (both ends outside the branch set), union-find in LDS (roots =
// smallest read id), labels, exact per-root counts, and, when one-read
// components cannot be eligible (min_reads >= 2), the component table in
// label order with each component's members grouped for the induce step.
// A listed read's local number is its tile's offset plus its slot in the
// tile, which orders local numbers like read ids, so the smaller local
// number is the smaller id.  A job with more listed reads (or mask tiles)
// than LDS holds uses the tagged global forest instead.  Largest jobs are
// dispatched first.
constexpr int kCcBlock = 1024;
constexpr int kCcCap = 16384;
constexpr int kCcPer = kCcCap / kCcBlock;
constexpr int kCcTileCap = 1024;
// jobs with more directed entries go through the single-graph kernels
constexpr int64_t kExternalEntries = 2 * (int64_t)kCcCap;
constexpr int32_t kNotEligible = -(1 << 30);

__device__ __forceinline__ int lds_find(int32_t *par, int x) {
  volatile int32_t *vp = par;
  while (true) {
    const int p = vp[x];
    if (p == x) return x;
    const int gp = vp[p];
    if (gp == p) return p;
    vp[x] = gp;  // path halving: gp is an ancestor of x
    x = gp;
  }
}

// link the larger root under the smaller one
__device__ __forceinline__ void lds_union(int32_t *par, int a, int b) {
  while (true) {
    a = lds_find(par, a);
    b = lds_find(par, b);
    if (a == b) return;
    const int hi = a > b ? a : b;
    const int lo = a > b ? b : a;
    if (atomicCAS(par + hi, hi, lo) == hi) return;
  }
}

__device__ __forceinline__ uint8_t kind_of(uint32_t c4) {
  return (c4 >> 2) == 1 ? CG_KIND_SINGLE : ((c4 & 3u) ? CG_KIND_PATH : CG_KIND_CYCLE);
}

__device__ void cc_global(const BatchDev &B, const BJob &J, int nt, const int2 *tc,
                          int64_t *sh64, int64_t *m_l_out);

__global__ __launch_bounds__(kCcBlock) void kb_cc_local(BatchDev B) {
  __shared__ int32_t s_par[kCcCap], s_aux[kCcCap];
  __shared__ int32_t s_pref[kCcTileCap + 1];
  __shared__ int64_t sh64[kCcBlock / kWave + 1];
  const int j = ld_const(B.job_order, blockIdx.x);
  const BJob J = job_at(B.jobs, j);
  if (J.external) return;
  const int nt = J.mt_count;
  const int tid = threadIdx.x;
  const bool table = J.min_reads >= 2;
  const int2 *tc = B.mt_cnt + J.mt_first;
  // listed reads per tile (prefix in LDS) and branch reads of the job
  int64_t L = 0, n_branch = 0;
  for (int base = 0; base < nt; base += kCcBlock) {
    const int t = base + tid;
    const int2 c = t < nt ? tc[t] : make_int2(0, 0);
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, kCcBlock>(((int64_t)c.y << 32) | c.x, sh64, &tot);
    if (t < nt && nt <= kCcTileCap) s_pref[t] = (int32_t)(L + (ex & 0xFFFFFFFF));
    L += tot & 0xFFFFFFFF;
    n_branch += tot >> 32;
  }
  if (tid == 0 && nt <= kCcTileCap) s_pref[nt] = (int32_t)L;
  __syncthreads();
  int64_t m_l = 0;
  if (L > 0 && (nt > kCcTileCap || L > kCcCap)) {
    cc_global(B, B.jobs[j], nt, tc, sh64, &m_l);
  } else if (L > 0) {
    // All of this thread's loads are issued before any is used, and every
    // global store waits for the tail: a barrier behind scattered stores
    // waits for them to land.
    const int per = (int)((L + kCcBlock - 1) / kCcBlock);
    const int l0 = tid * per;
    // 1. this thread's listed reads l0 .. l0 + per - 1: their slots in the
    // tiles' lists, their entries, then their neighbours' branch bits and
    // list slots
    int32_t slot[kCcPer];
    {
      int lo = 0, hi = nt - 1;  // tile of local number l0
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pref[mid] <= l0) lo = mid;
        else hi = mid - 1;
      }
      int t = lo;
#pragma unroll
      for (int k = 0; k < kCcPer; ++k) {
        const int l = l0 + k;
        slot[k] = -1;
        if (k < per && l < L) {
          while (s_pref[t + 1] <= l) ++t;
          slot[k] = t * kMaskTile + (l - s_pref[t]);
        }
      }
    }
    int4 e[kCcPer];
#pragma unroll
    for (int k = 0; k < kCcPer; ++k) e[k] = J.conn_list[slot[k] >= 0 ? slot[k] : 0];
    uint32_t fk[kCcPer];
    int32_t lu0[kCcPer], lu1[kCcPer];
#pragma unroll
    for (int k = 0; k < kCcPer; ++k) {
      const int l = l0 + k;
      fk[k] = 0;
      lu0[k] = lu1[k] = -1;
      if (slot[k] >= 0) {
        fk[k] = (uint32_t)e[k].w;
        s_aux[l] = e[k].x;
        s_par[l] = l;
        if (e[k].y >= 0) lu0[k] = s_pref[e[k].y / kMaskTile] + e[k].y % kMaskTile;
        if (e[k].z >= 0) lu1[k] = s_pref[e[k].z / kMaskTile] + e[k].z % kMaskTile;
        m_l += __popc(fk[k]);
      }
    }
    __syncthreads();
    // 2. union-find over local numbers (the larger root under the smaller)
#pragma unroll
    for (int k = 0; k < kCcPer; ++k) {
      if (lu0[k] >= 0) lds_union(s_par, l0 + k, lu0[k]);
      if (lu1[k] >= 0) lds_union(s_par, l0 + k, lu1[k]);
    }
    __syncthreads();
    int32_t r[kCcPer];
#pragma unroll
    for (int k = 0; k < kCcPer; ++k) r[k] = fk[k] ? lds_find(s_par, l0 + k) : l0 + k;
    __syncthreads();
    // 3. s_par becomes the per-root counter: 4 per read + 1 per path end
#pragma unroll
    for (int k = 0; k < kCcPer; ++k)
      if (slot[k] >= 0) s_par[l0 + k] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCcPer; ++k)
      if (fk[k]) atomicAdd(s_par + r[k], 4 + (__popc(fk[k]) == 1 ? 1 : 0));
    __syncthreads();
    int32_t c4[kCcPer];  // own roots' counts (a read without kept entries: 4)
    int32_t ne = 0, nq = 0;
#pragma unroll
    for (int k = 0; k < kCcPer; ++k) {
      const int l = l0 + k;
      c4[k] = 0;
      if (slot[k] >= 0) {
        if (!fk[k]) c4[k] = 4;
        else if (r[k] == l) c4[k] = s_par[l];
        if (table && fk[k] && r[k] == l && (c4[k] >> 2) >= J.min_reads) {
          ++ne;
          nq += c4[k] >> 2;
        }
      }
    }
    // 4. one scan: eligible roots, their reads and the kept entries (21 bits each)
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, kCcBlock>(
        ((int64_t)ne << 42) | ((int64_t)nq << 21) | m_l, sh64, &tot);
    const int64_t kMask21 = (1 << 21) - 1;
    if (table) {
      int32_t cb = (int32_t)(ex >> 42), mb = (int32_t)((ex >> 21) & kMask21);
      // s_par: member cursor of each eligible root, kNotEligible elsewhere
#pragma unroll
      for (int k = 0; k < kCcPer; ++k) {
        const int l = l0 + k;
        if (!fk[k] || r[k] != l) continue;
        const int32_t id = s_aux[l];
        if ((c4[k] >> 2) >= J.min_reads) {
          const int32_t q = c4[k] >> 2;
          J.parts.comp_label[cb] = id;
          J.parts.comp_size[cb] = q;
          J.parts.comp_kind[cb] = kind_of(c4[k]);
          J.parts.label_comp[id] = cb;
          J.s.memb[cb] = mb;
          J.s.comp_w[cb] = 0;
          s_par[l] = mb;
          ++cb;
          mb += q;
        } else {
          s_par[l] = kNotEligible;
        }
      }
      __syncthreads();
    }
    // 5. the tail: members, flags, labels, counts
#pragma unroll
    for (int k = 0; k < kCcPer; ++k) {
      if (!fk[k]) continue;
      const int32_t id = s_aux[l0 + k];
      J.flags[id] = (uint8_t)fk[k];
      J.label[id] = s_aux[r[k]];
      if (table) {
        const int32_t at = atomicAdd(s_par + r[k], 1);
        if (at >= 0) J.s.tmp[at] = id;
      } else {
        J.parts.label_comp[id] = c4[k];  // 0 for non-roots
      }
    }
    if (tid == 0) {
      if (table) *J.parts.d_n_comp = (int32_t)(tot >> 42);
      J.counts[0] = (int32_t)n_branch;
      J.counts[1] = (int32_t)(tot & kMask21);
    }
    return;
  }
  if (L == 0 && table && tid == 0) *J.parts.d_n_comp = 0;
  // BranchRemoval's counts: branch reads and kept entries
  int64_t tm;
  (void)block_excl_scan<int64_t, kCcBlock>(m_l, sh64, &tm);
  if (tid == 0) {
    J.counts[0] = (int32_t)n_branch;
    J.counts[1] = (int32_t)tm;
  }
}

// The same for a job beyond LDS: the job's own forest in global memory (only
// this workgroup touches it), the list walked tile by tile in id order.
__device__ void cc_global(const BatchDev &B, const BJob &J, int nt, const int2 *tc,
                          int64_t *sh64, int64_t *m_l_out) {
  const int tid = threadIdx.x;
  const uint32_t tag = forest_tag(B);
  const bool table = J.min_reads >= 2;
  uint32_t *lc = (uint32_t *)J.parts.label_comp;
  int64_t m_l = 0;
  // kept bits; counters of the reads with kept entries start at 0
  for (int t = 0; t < nt; ++t) {
    const int32_t c = tc[t].x;
    for (int i = tid; i < c; i += kCcBlock) {
      const int4 e = J.conn_list[t * kMaskTile + i];
      const uint32_t f = (uint32_t)e.w;
      if (f) {
        J.flags[e.x] = (uint8_t)f;
        lc[e.x] = 0;
      }
      m_l += __popc(f);
    }
  }
  *m_l_out = m_l;
  __syncthreads();
  for (int t = 0; t < nt; ++t) {
    const int32_t c = tc[t].x;
    for (int i = tid; i < c; i += kCcBlock) {
      const int4 e = J.conn_list[t * kMaskTile + i];
      if (e.y >= 0) tf_union(J.forest, tag, e.x, J.conn_list[e.y].x);
      if (e.z >= 0) tf_union(J.forest, tag, e.x, J.conn_list[e.z].x);
    }
  }
  __syncthreads();
  for (int t = 0; t < nt; ++t) {
    const int32_t c = tc[t].x;
    for (int i = tid; i < c; i += kCcBlock) {
      const int4 e = J.conn_list[t * kMaskTile + i];
      const uint32_t f = J.flags[e.x];
      if (!f) continue;
      int32_t r = e.x;
      while (true) {
        const int32_t p = tf_parent(J.forest, tag, r);
        if (p == r) break;
        r = p;
      }
      J.label[e.x] = r;
      atomicAdd(lc + r, 4u + (__popc(f) == 1 ? 1u : 0u));
    }
  }
  if (!table) return;
  __syncthreads();
  // component table in label order: the list in id order, chunk by chunk
  int32_t cb = 0, mb = 0;
  for (int t = 0; t < nt; ++t) {
    const int32_t c = tc[t].x;
    for (int base = 0; base < c; base += kCcBlock) {
      const int i = base + tid;
      int32_t id = -1;
      uint32_t c4 = 0;
      bool elig = false, root = false;
      if (i < c) {
        id = J.conn_list[t * kMaskTile + i].x;
        if (J.flags[id] & 6) {
          root = J.label[id] == id;
          if (root) {
            c4 = __hip_atomic_load(lc + id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            elig = (int32_t)(c4 >> 2) >= J.min_reads;
          }
        }
      }
      int64_t tot;
      const int64_t ex = block_excl_scan<int64_t, kCcBlock>(
          elig ? (((int64_t)1 << 32) | (c4 >> 2)) : 0, sh64, &tot);
      if (elig) {
        const int32_t k = cb + (int32_t)(ex >> 32);
        J.parts.comp_label[k] = id;
        J.parts.comp_size[k] = (int32_t)(c4 >> 2);
        J.parts.comp_kind[k] = kind_of(c4);
        J.s.memb[k] = mb + (int32_t)(ex & 0xFFFFFFFF);
        J.s.fill[k] = 0;
        J.s.comp_w[k] = 0;
      }
      if (i < c && (J.flags[id] & 6))
        __hip_atomic_store((int32_t *)lc + id, elig ? cb + (int32_t)(ex >> 32) : -1,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      cb += (int32_t)(tot >> 32);
      mb += (int32_t)(tot & 0xFFFFFFFF);
    }
  }
  if (tid == 0) *J.parts.d_n_comp = cb;
  __syncthreads();
  // members grouped by component
  for (int t = 0; t < nt; ++t) {
    const int32_t c = tc[t].x;
    for (int i = tid; i < c; i += kCcBlock) {
      const int32_t id = J.conn_list[t * kMaskTile + i].x;
      if (!(J.flags[id] & 6)) continue;
      const int32_t k = __hip_atomic_load((int32_t *)lc + J.label[id], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
      if (k < 0) continue;
      J.s.tmp[J.s.memb[k] + (int32_t)atomicAdd(J.s.fill + k, 1u)] = id;
    }
  }
}

// 3. eligible components in label order, reduce-then-scan: each tile counts
// its eligible roots, then each tile adds up the counts of the tiles before
// it in its job (plain loads, no waiting) and scatters
template <int T>
__device__ __forceinline__ bool eligible(const BJob &J, int64_t v, uint32_t *c_out) {
  if (v >= J.g.n) return false;
  const uint32_t c = (uint32_t)J.parts.label_comp[v];
  *c_out = c;
  const uint32_t mr = J.min_reads < 1 ? 1u : (uint32_t)J.min_reads;
  return (c >> 2) >= mr && !(J.flags[v] & 1);
}

template <int T>
__global__ __launch_bounds__(T) void kb_tilecount(BatchDev B) {
  __shared__ int32_t sh[T / kWave];
  const int t = blockIdx.x;
  const BJob J = job_at(B.jobs, ld_const(B.tile_job, t));
  if (J.min_reads >= 2 || J.external) return;  // table and members come from elsewhere
  const int64_t v = (int64_t)(t - J.vt_first) * T + threadIdx.x;
  uint32_t c = 0;
  const bool e = eligible<T>(J, v, &c);
  const int cnt = __popcll(__ballot(e));
  if (lane_id() == 0) sh[threadIdx.x / kWave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < T / kWave; ++w) s += sh[w];
    B.tile_cnt[t] = s;
  }
}

template <int T>
__global__ __launch_bounds__(T) void kb_compact(BatchDev B) {
  __shared__ int32_t sh[T / kWave + 1];
  const int t = blockIdx.x;
  const BJob J = job_at(B.jobs, ld_const(B.tile_job, t));
  if (J.min_reads >= 2 || J.external) return;  // table and members come from elsewhere
  int32_t before = 0;
  for (int i = J.vt_first + (int)threadIdx.x; i < t; i += T) before += B.tile_cnt[i];
  before = wave_sum(before);
  if (lane_id() == 0) sh[threadIdx.x / kWave] = before;
  __syncthreads();
  int32_t base = 0;
  for (int w = 0; w < T / kWave; ++w) base += sh[w];
  __syncthreads();
  const int64_t v = (int64_t)(t - J.vt_first) * T + threadIdx.x;
  uint32_t c = 0;
  const bool e = eligible<T>(J, v, &c);
  int32_t tot;
  const int32_t ex = base + block_excl_scan<int32_t, T>(e ? 1 : 0, sh, &tot);
  if (v < J.g.n) {
    if (e) {
      const uint32_t q = c >> 2;
      J.parts.comp_label[ex] = (int32_t)v;
      J.parts.comp_size[ex] = (int32_t)q;
      J.parts.comp_kind[ex] = q == 1 ? CG_KIND_SINGLE : ((c & 3u) ? CG_KIND_PATH : CG_KIND_CYCLE);
      J.parts.label_comp[v] = ex;
      J.s.comp_w[ex] = 0;
    } else {
      J.parts.label_comp[v] = -1;
    }
  }
  if (t == J.vt_first + J.vt_count - 1 && threadIdx.x == 0) *J.parts.d_n_comp = base + tot;
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
// per-chunk setup too often.
constexpr int kChunkPieces = 32;
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
    for (int c = threadIdx.x; c < nc; c += kBatchLptBlock) J.s.fill[c] = 0;
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
    xh += (xp + kChunkPieces - 1) / kChunkPieces;
  }
  int64_t tcp, th;
  int64_t ecp = block_excl_scan<int64_t, kBatchLptBlock>(xcp, sh, &tcp);
  int64_t eh = block_excl_scan<int64_t, kBatchLptBlock>(xh, sh, &th);
  for (int i = i0; i < i1; ++i) {
    const uint64_t w = __hip_atomic_load((uint64_t *)(B.job_cnt + i), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    const int64_t xc = (int32_t)(uint32_t)w, xp = (int32_t)(uint32_t)(w >> 32);
    B.comp_base[i] = (int32_t)(ecp >> 32);
    B.piece_base[i] = (int32_t)(uint32_t)ecp;
    B.chunk_base[i] = (int32_t)eh;
    ecp += (xc << 32) | xp;
    eh += (xp + kChunkPieces - 1) / kChunkPieces;
  }
  if (threadIdx.x == 0) {
    B.comp_base[B.n_jobs] = (int32_t)(tcp >> 32);
    B.piece_base[B.n_jobs] = (int32_t)(uint32_t)tcp;
    B.chunk_base[B.n_jobs] = (int32_t)th;
    B.counters[2] = 0;
    B.counters[3] += 1u;  // the next run's forest tag
  }
  __threadfence();
}

// 4b. the job of every batch-wide component and copy chunk, so that the
// persistent passes find it with one load: one entry per thread, by binary
// search in the bases (staged in LDS up to kTablesJobCap jobs)
constexpr int kTablesBlock = 256;
constexpr int kTablesJobCap = 4096;

__global__ __launch_bounds__(kTablesBlock) void kb_tables(BatchDev B) {
  __shared__ int32_t s_cb[kTablesJobCap + 1], s_hb[kTablesJobCap + 1];
  __shared__ int32_t s_hist[kWqBuckets];
  for (int b = threadIdx.x; b < kWqBuckets; b += kTablesBlock) s_hist[b] = 0;
  const int nj = B.n_jobs;
  const bool in_lds = nj <= kTablesJobCap;
  if (in_lds) {
    for (int i = threadIdx.x; i <= nj; i += kTablesBlock) {
      s_cb[i] = B.comp_base[i];
      s_hb[i] = B.chunk_base[i];
    }
  }
  __syncthreads();
  const int32_t tc = B.comp_base[nj], th = B.chunk_base[nj];
  const int32_t nmax = tc > th ? tc : th;
  for (int32_t i = blockIdx.x * kTablesBlock + threadIdx.x; i < nmax;
       i += gridDim.x * kTablesBlock) {
    if (i < tc) {
      const int j = job_of(in_lds ? s_cb : B.comp_base, nj, i);
      B.comp_job[i] = j;
      // the work queue's histogram: components per read count
      const int32_t q = B.jobs[j].parts.comp_size[i - (in_lds ? s_cb[j] : B.comp_base[j])];
      atomicAdd(s_hist + (q < kWqBuckets - 1 ? q : kWqBuckets - 1), 1);
    }
    if (i < th) B.chunk_job[i] = job_of(in_lds ? s_hb : B.chunk_base, nj, i);
  }
  // (counted in LDS: many components share a read count, and their global
  // atomics would queue on one address)
  __syncthreads();
  for (int b = threadIdx.x; b < kWqBuckets; b += kTablesBlock)
    if (s_hist[b]) atomicAdd(B.wq_hist + b, s_hist[b]);
}

// 4c. the work queue: every component of the batch in decreasing read count
// (within a bucket in any order), as (job, component, reads, first local
// number), and the queue heads of the four per-component passes.  Handing
// the largest components out first to whichever workgroup is free is LPT
// list scheduling of the whole batch's components onto the workgroups.
// Components of at most kWalkSmallCap (kIndSmallCap) reads form the queue's
// tail, which the one-wave passes take.
constexpr int kWqBlock = 256;
constexpr int kWqPer = kWqBuckets / kWqBlock;

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
    B.wq_meta[2] = s_start[kIndSmallCap];   // above kIndSmallCap
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
  int4 first = make_int4(-1, 0, 0, 0);
  for (int32_t i = i0 + threadIdx.x; i < i1; i += kWqBlock) {
    const int j = B.comp_job[i];
    const int32_t c = i - B.comp_base[j];
    const cg_parts &P = B.jobs[j].parts;
    const int32_t q = P.comp_size[c];
    if (i == i0 + (int32_t)threadIdx.x) first = make_int4(j, c, q, P.comp_start[c]);
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
    int4 e = first;
    if (i != i0 + (int32_t)threadIdx.x) {
      const int j = B.comp_job[i];
      const int32_t c = i - B.comp_base[j];
      const cg_parts &P = B.jobs[j].parts;
      e = make_int4(j, c, P.comp_size[c], P.comp_start[c]);
    }
    const int b = e.z < kWqBuckets - 1 ? e.z : kWqBuckets - 1;
    B.wq[s_base[b] + atomicAdd(s_cnt + b, 1)] = e;
  }
}

// 5. each eligible read claims a slot in its component's block
template <int T>
__global__ __launch_bounds__(T) void kb_fill(BatchDev B) {
  const int t = blockIdx.x;
  const BJob J = job_at(B.jobs, ld_const(B.tile_job, t));
  if (J.min_reads >= 2 || J.external) return;  // table and members come from elsewhere
  const int64_t v = (int64_t)(t - J.vt_first) * T + threadIdx.x;
  if (v >= J.g.n) return;
  const int32_t c = J.parts.label_comp[J.label[v]];
  if (c < 0) return;
  const uint32_t slot = atomicAdd(J.s.fill + c, 1u);
  J.s.tmp[J.parts.comp_start[c] + slot] = (int32_t)v;
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

// 6. induced subgraph of each component: sorted local numbers and local CSR
// rows
template <int BLOCK, int CAP>
__device__ __forceinline__ void induce_listed(const BatchDev &B, int4 d, int32_t *a,
                                              int32_t *sh_scan) {
  // d = (job, component, reads, first local number), uniform
  const int j = __builtin_amdgcn_readfirstlane(d.x), c = __builtin_amdgcn_readfirstlane(d.y);
  const int q = __builtin_amdgcn_readfirstlane(d.z), st = __builtin_amdgcn_readfirstlane(d.w);
  const BJob J = job_at(B.jobs, j);
  const int32_t *members = J.s.tmp + (J.min_reads >= 2 ? J.s.memb[c] : st);
  induce_component<BLOCK, CAP>(q, st, J.s.estart[c], members, J.flags, J.g.row_ptr, J.g.col,
                               J.local.perm, J.s.lidx, J.local.loc_row_ptr, J.local.loc_col,
                               J.local.loc_eid, a, sh_scan);
}

// 6a. components of at most kIndSmallCap reads (the queue's tail): one wave each
__global__ __launch_bounds__(kIndSmallBlock) void kb_induce_small(BatchDev B) {
  __shared__ int32_t a[kIndSmallCap];
  __shared__ int32_t sh_scan[kIndSmallBlock / kWave + 1];
  const int32_t lo = ld_const(B.wq_meta, 2), hi = ld_const(B.wq_meta, 0);
  for (int32_t r = 0, x; (x = wq_entry(lo, hi, r)) >= 0; ++r)
    induce_listed<kIndSmallBlock, kIndSmallCap>(B, wq_at(B, x), a, sh_scan);
}

// 6b. the larger components (the queue's head, largest first)
__global__ __launch_bounds__(kIndBlock) void kb_induce(BatchDev B) {
  __shared__ int32_t a[kIndLocalCap];
  __shared__ int32_t sh_scan[kIndBlock / kWave + 1];
  const int32_t hi = ld_const(B.wq_meta, 2);
  for (int32_t r = 0, x; (x = wq_entry(0, hi, r)) >= 0; ++r)
    induce_listed<kIndBlock, kIndLocalCap>(B, wq_at(B, x), a, sh_scan);
}

// 7. walk every component
// 7a. components of at most kWalkSmallCap reads (the queue's tail): one wave each
__global__ __launch_bounds__(kWalkSmallBlock) void kb_walk_small(BatchDev B) {
  __shared__ int32_t s_nb[2 * kWalkSmallCap], s_eid[2 * kWalkSmallCap], s_nxt[2 * kWalkSmallCap],
      s_dist[2 * kWalkSmallCap], s_endv[2 * kWalkSmallCap], s_vid[kWalkSmallCap];
  __shared__ uint32_t s_rlen[kWalkSmallCap], s_eo[2 * kWalkSmallCap], s_ep[2 * kWalkSmallCap];
  __shared__ uint8_t s_es[2 * kWalkSmallCap];
  __shared__ uint32_t sh_scan[kWalkSmallBlock / kWave + 1];
  const int32_t lo = ld_const(B.wq_meta, 1), hi = ld_const(B.wq_meta, 0);
  for (int32_t r = 0, x; (x = wq_entry(lo, hi, r)) >= 0; ++r) {
    const int4 d = wq_at(B, x);
    const BJob J = job_at(B.jobs, d.x);
    WalkArrays w{s_nb, s_eid, s_nxt, s_dist, s_endv, s_vid, s_rlen, s_es, s_eo, s_ep};
    walk_component<kWalkSmallBlock, kWalkSmallCap, true>(
        d.y, d.z, d.w, w, J.g, J.parts, J.local.perm, J.local.loc_row_ptr, J.local.loc_col,
        J.local.loc_eid, J.out, J.s, nullptr, sh_scan);
  }
}

// 7b. the larger components (the queue's head, largest first)
__global__ __launch_bounds__(kWalkBlock) void kb_walk(BatchDev B) {
  __shared__ int32_t s_nb[2 * kWalkCap], s_eid[2 * kWalkCap], s_nxt[2 * kWalkCap],
      s_dist[2 * kWalkCap], s_endv[2 * kWalkCap], s_vid[kWalkCap];
  __shared__ uint32_t s_rlen[kWalkCap], s_eo[2 * kWalkCap], s_ep[2 * kWalkCap];
  __shared__ uint8_t s_es[2 * kWalkCap];
  __shared__ uint32_t sh_scan[kWalkBlock / kWave + 1];
  const int32_t hi = ld_const(B.wq_meta, 1);
  for (int32_t r = 0, x; (x = wq_entry(0, hi, r)) >= 0; ++r) {
    const int4 d = wq_at(B, x);
    const int c = d.y, q = d.z, st = d.w;
    const BJob J = job_at(B.jobs, d.x);
    if (q <= kWalkCap) {
      WalkArrays w{s_nb, s_eid, s_nxt, s_dist, s_endv, s_vid, s_rlen, s_es, s_eo, s_ep};
      walk_component<kWalkBlock, kWalkCap, true>(c, q, st, w, J.g, J.parts, J.local.perm,
                                                 J.local.loc_row_ptr, J.local.loc_col,
                                                 J.local.loc_eid, J.out, J.s, nullptr, sh_scan);
    } else {
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
}

// 8. contig word offsets per job
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
}

// 9. packed copy: one wave per chunk of kChunkPieces consecutive pieces of a
// job (the grid covers an upper bound on the chunks; waves past the last exit)
__device__ __forceinline__ PieceArrays piece_arrays(const BJob &J) {
  return piece_arrays(J.s.lay_contig, J.out.layout_vid, J.out.layout_rev, J.s.piece_off,
                      J.s.piece_len, J.s.piece_skip, J.g.read_off, J.g.read_len, J.out.len,
                      J.out.base_off);
}

__global__ __launch_bounds__(1024) void kb_copy(BatchDev B) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t gw = blockIdx.x * (blockDim.x / kWave) + wave;
  const int32_t nwv = gridDim.x * (blockDim.x / kWave);
  const int32_t total = ld_const(B.chunk_base, B.n_jobs);
  for (int32_t ch = gw; ch < total; ch += nwv) {
    // a chunk never spans two jobs, so the job is the same for the whole wave
    const int j = ld_const(B.chunk_job, ch);
    const BJob J = job_at(B.jobs, j);
    if (*J.out.d_total_words > J.out.cap_words) continue;
    const int32_t n_e = ld_const(B.piece_base, j + 1) - ld_const(B.piece_base, j);
    const int32_t c0 = (ch - ld_const(B.chunk_base, j)) * kChunkPieces;
    const int cnt = n_e - c0 < kChunkPieces ? n_e - c0 : kChunkPieces;
    copy_chunk(J.g.seq, J.g.seq_words, J.out.bases, piece_arrays(J), c0, cnt, n_e, lane_id());
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
  bool any_single;  // a job with min_reads <= 1 (one-read components eligible)
  bool any_bases;   // a job partitioned by bases weights
  int64_t chunk_slots;  // upper bound on the copy chunks of the batch
  // workgroups of each per-component pass that fit on the device at once:
  // their grids stay within it, so every workgroup of the snake order runs
  // from the start (a workgroup that waits for a free slot starts its whole
  // share late)
  int res_induce_small, res_induce, res_walk_small, res_walk;
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
};

static int check_job(const cg_job &J, int i) {
  const cg_graph &g = J.g;
  if (g.n < 0 || g.n >= (1 << 30) || g.m < 0 || !g.row_ptr ||
      (g.m > 0 && (!g.col || !g.ovl || !g.strand)) ||
      (g.n > 0 && (!g.read_len || !g.read_off || !g.seq)) || ((g.pre == nullptr) != (g.post == nullptr)))
    return set_error(CG_EINVAL, "job %d: bad graph", i);
  if (J.P < 1 || J.P > 65536) return set_error(CG_EINVAL, "job %d: P=%d outside [1, 65536]", i, J.P);
  if (J.weight != CG_WEIGHT_READS && J.weight != CG_WEIGHT_BASES)
    return set_error(CG_EINVAL, "job %d: weight=%d", i, J.weight);
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
  // the mask pass moves four reads per thread with 16-byte accesses
  if (((uintptr_t)g.row_ptr & 15) || ((uintptr_t)J.label & 15) || ((uintptr_t)p.label_comp & 15) ||
      ((uintptr_t)J.flags & 3))
    return set_error(CG_EINVAL,
                     "job %d: row_ptr, label and label_comp must be 16-byte aligned and flags "
                     "4-byte aligned", i);
  return CG_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <int T>
static void launch_vertex_phases(cg_batch *b, hipStream_t st) {
  cg_ctx *ctx = b->ctx;
  const BatchDev &B = b->dev;
  CG_LAUNCH(ctx, kb_tilecount<T>, dim3(b->n_vtiles), dim3(T), st, B);
  CG_LAUNCH(ctx, kb_compact<T>, dim3(b->n_vtiles), dim3(T), st, B);
}

template <int T>
static void launch_vertex_fill(cg_batch *b, hipStream_t st) {
  cg_ctx *ctx = b->ctx;
  CG_LAUNCH(ctx, kb_fill<T>, dim3(b->n_vtiles), dim3(T), st, b->dev);
}

extern "C" {

int cg_batch_create(cg_ctx *ctx, int32_t n_jobs, const cg_job *jobs,
                    const cg_batch_params *params, cg_batch **out) {
  if (!ctx || !jobs || !out || n_jobs < 1) return set_error(CG_EINVAL, "bad batch arguments");
  *out = nullptr;
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
  int64_t total_n = 0;
  for (int i = 0; i < n_jobs; ++i) {
    int rc = check_job(jobs[i], i);
    if (rc) return rc;
    total_n += jobs[i].g.n + 1;
  }
  if (total_n >= (1ll << 31)) return set_error(CG_EUNSUPPORTED, "batch holds 2^31 or more reads");
  const int T = prm.vertex_tile;
  std::vector<BJob> hj(n_jobs);
  std::vector<int32_t> tile_job;
  std::vector<size_t> job_off(n_jobs);
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t here = at;
    at += align256(bytes);
    return here;
  };
  const size_t o_jobs = take(sizeof(BJob) * n_jobs);
  int32_t nv = 0;
  for (int i = 0; i < n_jobs; ++i) {
    const int32_t cnt = (int32_t)((jobs[i].g.n + 1 + T - 1) / T);
    hj[i].vt_first = nv;
    hj[i].vt_count = cnt;
    for (int32_t t = 0; t < cnt; ++t) tile_job.push_back(i);
    nv += cnt;
  }
  const size_t o_tiles = take(sizeof(int32_t) * nv);
  const size_t o_tcnt = take(sizeof(int32_t) * nv);
  const size_t o_cbase = take(sizeof(int32_t) * (n_jobs + 1));
  const size_t o_pbase = take(sizeof(int32_t) * (n_jobs + 1));
  const size_t o_hbase = take(sizeof(int32_t) * (n_jobs + 1));
  const size_t o_jcnt = take(sizeof(int2) * (n_jobs > 0 ? n_jobs : 1));
  int64_t sum_n = 0, sum_chunks = 0;
  for (int i = 0; i < n_jobs; ++i) {
    sum_n += jobs[i].g.n;
    sum_chunks += (jobs[i].g.n + kChunkPieces - 1) / kChunkPieces;
  }
  const size_t o_cjob = take(sizeof(int32_t) * (size_t)(sum_n > 0 ? sum_n : 1));
  const size_t o_wq = take(sizeof(int4) * (size_t)(sum_n > 0 ? sum_n : 1));
  const size_t o_wqh = take(sizeof(int32_t) * kWqBuckets);
  const size_t o_wqc = take(sizeof(int32_t) * kWqBuckets);
  const size_t o_wqm = take(sizeof(int32_t) * 8);
  const size_t o_hjob = take(sizeof(int32_t) * (size_t)(sum_chunks > 0 ? sum_chunks : 1));
  const size_t o_counters = take(sizeof(unsigned int) * 8);
  const size_t o_order = take(sizeof(int32_t) * n_jobs);
  int32_t n_mt = 0;
  for (int i = 0; i < n_jobs; ++i) {
    // a job whose reads of degree 1-2 (about half its entries) would not fit
    // the components pass's LDS goes through the single-graph kernels
    hj[i].external = jobs[i].g.m > kExternalEntries ? 1 : 0;
    hj[i].mt_first = n_mt;
    hj[i].mt_count = hj[i].external ? 0 : (jobs[i].g.n + kMaskTile - 1) / kMaskTile;
    n_mt += hj[i].mt_count;
  }
  const size_t o_mtiles = take(sizeof(MaskTile) * (n_mt > 0 ? n_mt : 1));
  const size_t o_mtcnt = take(sizeof(int2) * (n_mt > 0 ? n_mt : 1));
  std::vector<size_t> forest_off(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    job_off[i] = take(layout(jobs[i].g.n, jobs[i].g.m, jobs[i].P).total);
    forest_off[i] = take(sizeof(uint64_t) * (size_t)(jobs[i].g.n > 0 ? jobs[i].g.n : 1));
  }
  cg_batch *b = new (std::nothrow) cg_batch();
  if (!b) return set_error(CG_EINVAL, "out of host memory");
  b->ctx = ctx;
  b->n_jobs = n_jobs;
  b->n_vtiles = nv;
  b->chunk_slots = sum_chunks;
  b->any_single = false;
  b->any_bases = false;
  for (int i = 0; i < n_jobs; ++i) {
    b->any_single |= jobs[i].min_reads < 2;
    b->any_bases |= jobs[i].weight == CG_WEIGHT_BASES;
  }
  b->prm = prm;
  {
    int dev = 0, cus = 0, k1 = 0, k2 = 0, k3 = 0, k4 = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&k1, kb_induce_small, kIndSmallBlock, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&k2, kb_induce, kIndBlock, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&k3, kb_walk_small, kWalkSmallBlock, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&k4, kb_walk, kWalkBlock, 0) != hipSuccess) {
      delete b;
      return set_error(CG_EHIP, "occupancy query failed");
    }
    b->res_induce_small = k1 * cus;
    b->res_induce = k2 * cus;
    b->res_walk_small = k3 * cus;
    b->res_walk = k4 * cus;
  }
  b->mem_bytes = at;
  b->mem = nullptr;
  b->graph = nullptr;
  b->exec = nullptr;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  int rc = hip_check(hipMalloc((void **)&b->mem, at), "hipMalloc(batch)");
  if (!rc) rc = hip_check(hipMemset(b->mem, 0, at), "hipMemset(batch)");
  if (!rc) {
    for (int i = 0; i < n_jobs; ++i) {
      const cg_job &J = jobs[i];
      BJob &h = hj[i];
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
      // carve this job's scratch slice the way a context carves its scratch
      cg_ctx view{};
      view.scratch = b->mem + job_off[i];
      view.scratch_bytes = layout(J.g.n, J.g.m, J.P).total;
      carve(&view, J.g.n, J.g.m, J.P, &h.s);
      // zeroed above: tag 0 never matches a run's tag (runs use 1, 2, ...)
      h.forest = (uint64_t *)(b->mem + forest_off[i]);
      // the list and its index live in scratch that later steps reuse
      h.conn_list = (int4 *)h.s.walk;
      h.conn_map = h.s.lidx;
      if (h.external) {
        b->ext_jobs.push_back(J);
        b->ext_s.push_back(h.s);
      }
    }
    std::vector<MaskTile> mt;
    mt.reserve(n_mt);
    int2 *d_mtcnt = (int2 *)(b->mem + o_mtcnt);
    for (int i = 0; i < n_jobs; ++i)
      for (int32_t v0 = 0; !hj[i].external && v0 < jobs[i].g.n; v0 += kMaskTile)
        mt.push_back(MaskTile{jobs[i].g.row_ptr, jobs[i].g.col, jobs[i].flags, jobs[i].label,
                              jobs[i].parts.label_comp, hj[i].conn_list, hj[i].conn_map,
                              d_mtcnt + (int32_t)mt.size(), jobs[i].g.n, v0,
                              jobs[i].min_reads >= 2 ? -1 : 4});
    std::vector<int32_t> order(n_jobs);
    for (int i = 0; i < n_jobs; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return jobs[a].g.n > jobs[c].g.n; });
    if (n_mt > 0)
      rc = hip_check(hipMemcpy(b->mem + o_mtiles, mt.data(), sizeof(MaskTile) * n_mt,
                               hipMemcpyHostToDevice), "hipMemcpy(mask tiles)");
    if (!rc)
      rc = hip_check(hipMemcpy(b->mem + o_order, order.data(), sizeof(int32_t) * n_jobs,
                               hipMemcpyHostToDevice), "hipMemcpy(job order)");
  }
  if (!rc) {
    rc = hip_check(hipMemcpy(b->mem + o_jobs, hj.data(), sizeof(BJob) * n_jobs,
                             hipMemcpyHostToDevice), "hipMemcpy(jobs)");
  }
  if (!rc)
    rc = hip_check(hipMemcpy(b->mem + o_tiles, tile_job.data(), sizeof(int32_t) * nv,
                             hipMemcpyHostToDevice), "hipMemcpy(tiles)");
  (void)hipSetDevice(prev);
  if (rc) {
    if (b->mem) (void)hipFree(b->mem);
    delete b;
    return rc;
  }
  BatchDev &d = b->dev;
  d.jobs = (BJob *)(b->mem + o_jobs);
  d.tile_job = (int32_t *)(b->mem + o_tiles);
  d.tile_cnt = (int32_t *)(b->mem + o_tcnt);
  d.comp_base = (int32_t *)(b->mem + o_cbase);
  d.piece_base = (int32_t *)(b->mem + o_pbase);
  d.chunk_base = (int32_t *)(b->mem + o_hbase);
  d.job_cnt = (int2 *)(b->mem + o_jcnt);
  d.wq = (int4 *)(b->mem + o_wq);
  d.wq_hist = (int32_t *)(b->mem + o_wqh);
  d.wq_cur = (int32_t *)(b->mem + o_wqc);
  d.wq_meta = (int32_t *)(b->mem + o_wqm);
  d.comp_job = (int32_t *)(b->mem + o_cjob);
  d.chunk_job = (int32_t *)(b->mem + o_hjob);
  d.counters = (unsigned int *)(b->mem + o_counters);
  d.mt_cnt = (int2 *)(b->mem + o_mtcnt);
  d.job_order = (const int32_t *)(b->mem + o_order);
  d.mtiles = (const MaskTile *)(b->mem + o_mtiles);
  d.n_mtiles = n_mt;
  d.fixed = ctx->fixed;
  d.n_jobs = n_jobs;
  d.n_vtiles = nv;
  *out = b;
  return CG_OK;
}

int cg_batch_run(cg_batch *b, void *stream) {
  if (!b) return set_error(CG_EINVAL, "batch is NULL");
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
  if (B.n_mtiles > 0) {
    CG_LAUNCH(ctx, kb_mask_list, dim3(B.n_mtiles), dim3(kMaskThreads), st, B.mtiles);
    CG_LAUNCH(ctx, kb_cc_prep, dim3(B.n_mtiles), dim3(kMaskThreads), st, B.mtiles);
  }
  CG_LAUNCH(ctx, kb_cc_local, dim3(b->n_jobs), dim3(kCcBlock), st, B);
  // jobs where one-read components are eligible take their component table
  // and member buckets from full vertex passes
  if (b->any_single) {
    if (T == 256) launch_vertex_phases<256>(b, st);
    else if (T == 512) launch_vertex_phases<512>(b, st);
    else launch_vertex_phases<1024>(b, st);
  }
  if (b->any_bases) {
    if (T == 256) CG_LAUNCH(ctx, kb_weight<256>, dim3(b->n_vtiles), dim3(256), st, B);
    else if (T == 512) CG_LAUNCH(ctx, kb_weight<512>, dim3(b->n_vtiles), dim3(512), st, B);
    else CG_LAUNCH(ctx, kb_weight<1024>, dim3(b->n_vtiles), dim3(1024), st, B);
  }
  CG_LAUNCH(ctx, kb_lpt, dim3(b->n_jobs), dim3(kBatchLptBlock), st, B);
  CG_LAUNCH(ctx, kb_tables, dim3(256), dim3(kTablesBlock), st, B);
  CG_LAUNCH(ctx, kb_wq_place, dim3(128), dim3(kWqBlock), st, B);
  if (b->any_single) {
    if (T == 256) launch_vertex_fill<256>(b, st);
    else if (T == 512) launch_vertex_fill<512>(b, st);
    else launch_vertex_fill<1024>(b, st);
  }
  auto capped = [](int want, int fit) { return dim3((unsigned)(fit > 0 && fit < want ? fit : want)); };
  CG_LAUNCH(ctx, kb_induce_small, capped(4 * PB, b->res_induce_small), dim3(kIndSmallBlock), st, B);
  CG_LAUNCH(ctx, kb_induce, capped(PB, b->res_induce), dim3(kIndBlock), st, B);
  CG_LAUNCH(ctx, kb_walk_small, capped(4 * PB, b->res_walk_small), dim3(kWalkSmallBlock), st, B);
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
