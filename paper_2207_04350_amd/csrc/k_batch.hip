// Batched form: the five steps of Algorithm 2 for many independent string
// graphs ("jobs") with one launch per phase for the whole batch.
//
//  vertex passes   each job is cut into tiles of T vertices; a launch covers
//                  the tiles of every job (tile -> job table)
//  compaction      reduce-then-scan per job: tiles count, then each tile adds
//                  up the counts of the tiles before it in its job
//  component and   persistent grids stride over the batch-wide item ranges
//  piece passes    (components, pieces) whose per-job bases the last LPT
//                  workgroup computes on the device
//
// Every counter a launch uses is reset by the launch itself, and the
// union-find forest is reset by bumping its tag, so the ten launches can be
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
  int32_t P, min_reads;
  uint8_t *flags;
  int32_t *counts;
  int32_t *label;
  cg_parts parts;
  cg_local local;
  cg_contigs out;
  Scratch s;
  uint64_t *forest;            // [n] tagged union-find forest (batch-owned, never reused)
  int4 *conn_list;             // [n] reads with kept entries: (id, kept neighbours or -1, flags),
                               // each mask tile's reads packed at the start of its slice
  int32_t *conn_map;           // [n] slot of a read in conn_list
  int32_t vt_first, vt_count;  // the job's vertex tiles (covering 0..n)
  int32_t mt_first, mt_count;  // the job's mask tiles
};

// One tile of the mask pass: kMaskTile consecutive reads of one job.
struct MaskTile {
  const int32_t *row_ptr;
  const int32_t *col;
  uint8_t *flags;
  int32_t *label;
  int32_t *label_comp;
  int4 *conn_list;
  int32_t *conn_map;
  int32_t *conn_cnt;  // this tile's number of listed reads
  int32_t n, v0;
};
constexpr int kMaskThreads = 256;
constexpr int kMaskTile = 4 * kMaskThreads;

struct BatchDev {
  BJob *jobs;                       // [n_jobs]
  int32_t *tile_job;                // [n_vtiles]
  int32_t *tile_cnt;                // [n_vtiles] eligible roots per tile
  int32_t *comp_base;               // [n_jobs + 1] first component item of each job
  int32_t *piece_base;              // [n_jobs + 1] first piece item of each job
  int32_t *chunk_base;              // [n_jobs + 1] first 64-piece copy chunk of each job
  unsigned int *counters;           // [8] 2: LPT ticket, 3: runs so far (forest tag - 1)
  int32_t *mt_conn;                 // [n_mtiles] listed reads of each mask tile
  const int32_t *job_order;         // [n_jobs] jobs by decreasing read count
  const MaskTile *mtiles;           // [n_mtiles]
  Fixed *fixed;
  int32_t n_jobs, n_vtiles, n_mtiles;
};

// index j with base[j] <= i < base[j+1] (base ascending, base[0] = 0)
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
// 1. mask (four reads per thread, 16-byte loads and stores): branch flags and
// kept entries, labels and size counters initialised (a read without kept
// entries is its own one-read component: label = id, count final here), and
// every read with kept entries listed with its kept neighbours.  The branch /
// kept-entry counts are summed later by the job's LPT workgroup.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t forest_tag(const BatchDev &B) { return B.counters[3] + 1u; }

__device__ __forceinline__ int32_t deg_of(const int32_t *__restrict__ row_ptr, int32_t u) {
  return row_ptr[u + 1] - row_ptr[u];
}

__global__ __launch_bounds__(kMaskThreads) void kb_mask_list(const MaskTile *__restrict__ tiles) {
  const MaskTile D = tiles[blockIdx.x];
  const int32_t n = D.n;
  const int32_t v0 = D.v0 + 4 * (int32_t)threadIdx.x;
  const int lane = lane_id();
  // row_ptr[v0 .. v0+4]
  int4 a = make_int4(0, 0, 0, 0);
  if (v0 + 3 <= n) {
    a = *(const int4 *)(D.row_ptr + v0);
  } else if (v0 <= n) {
    a.x = D.row_ptr[v0];
    if (v0 + 1 <= n) a.y = D.row_ptr[v0 + 1];
    if (v0 + 2 <= n) a.z = D.row_ptr[v0 + 2];
  }
  int32_t e4 = __shfl_down(a.x, 1);
  if (lane == kWave - 1 && v0 + 4 <= n) e4 = D.row_ptr[v0 + 4];
  const int32_t rp[5] = {a.x, a.y, a.z, a.w, e4};
  // kept entries: the rows of degree 1-2 read their columns, then the
  // neighbours' degrees (all loads issued before any is used)
  int32_t u0[4], u1[4], dg[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool live = v0 + i < n;
    dg[i] = live ? rp[i + 1] - rp[i] : 0;
    u0[i] = (dg[i] == 1 || dg[i] == 2) ? D.col[rp[i]] : -1;
    u1[i] = dg[i] == 2 ? D.col[rp[i] + 1] : -1;
  }
  int32_t d0[4], d1[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    d0[i] = u0[i] >= 0 ? deg_of(D.row_ptr, u0[i]) : 3;
    d1[i] = u1[i] >= 0 ? deg_of(D.row_ptr, u1[i]) : 3;
  }
  uint32_t f[4];
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f[i] = dg[i] >= 3 ? 1u : ((d0[i] < 3 ? 2u : 0u) | (d1[i] < 3 ? 4u : 0u));
    cnt += (f[i] & 6) ? 1 : 0;
  }
  if (v0 + 3 < n) {
    *(uint32_t *)(D.flags + v0) = f[0] | (f[1] << 8) | (f[2] << 16) | (f[3] << 24);
    *(int4 *)(D.label + v0) = make_int4(v0, v0 + 1, v0 + 2, v0 + 3);
    *(int4 *)(D.label_comp + v0) = make_int4((f[0] & 6) ? 0 : 4, (f[1] & 6) ? 0 : 4,
                                             (f[2] & 6) ? 0 : 4, (f[3] & 6) ? 0 : 4);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (v0 + i < n) {
        D.flags[v0 + i] = (uint8_t)f[i];
        D.label[v0 + i] = v0 + i;
        D.label_comp[v0 + i] = (f[i] & 6) ? 0 : 4;
      }
  }
  // the tile's reads with kept entries, packed in id order at the start of
  // the tile's slice of the list (a block scan, no global atomics)
  __shared__ int32_t sh[kMaskThreads / kWave + 1];
  int32_t tot;
  int32_t pos = D.v0 + block_excl_scan<int32_t, kMaskThreads>(cnt, sh, &tot);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (f[i] & 6) {
      D.conn_list[pos] = make_int4(v0 + i, (f[i] & 2) ? u0[i] : -1, (f[i] & 4) ? u1[i] : -1,
                                   (int32_t)f[i]);
      D.conn_map[v0 + i] = pos;
      ++pos;
    }
  if (threadIdx.x == 0) *D.conn_cnt = tot;
}

// 2. components of each job in one workgroup: union-find in LDS over the
// job's listed reads (roots = smallest read id, exact per-root counts, no
// global atomics).  A listed read's local number is its tile's offset plus
// its slot in the tile, which orders local numbers like read ids, so the
// smaller local number is the smaller id.  A job with more listed reads (or
// mask tiles) than LDS holds uses the tagged global forest instead.  Largest
// jobs are dispatched first.
constexpr int kCcBlock = 1024;
constexpr int kCcCap = 16384;
constexpr int kCcPer = kCcCap / kCcBlock;
constexpr int kCcTileCap = 1024;

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

__global__ __launch_bounds__(kCcBlock) void kb_cc_local(BatchDev B) {
  __shared__ int32_t s_par[kCcCap];
  __shared__ int32_t s_pref[kCcTileCap + 1];
  __shared__ int32_t sh[kCcBlock / kWave + 1];
  const int j = B.job_order[blockIdx.x];
  const BJob &J = B.jobs[j];
  const int nt = J.mt_count;
  if (nt == 0) return;
  const int32_t *cnt = B.mt_conn + J.mt_first;
  const int4 *__restrict__ list = J.conn_list;
  const int32_t *__restrict__ map = J.conn_map;
  const int tid = threadIdx.x;
  if (nt <= kCcTileCap) {
    int32_t tot;
    const int32_t c = tid < nt ? cnt[tid] : 0;
    const int32_t ex = block_excl_scan<int32_t, kCcBlock>(c, sh, &tot);
    if (tid < nt) s_pref[tid] = ex;
    if (tid == 0) s_pref[nt] = tot;
    __syncthreads();
    const int32_t L = tot;
    if (L == 0) return;
    if (L <= kCcCap) {
      // slot of local number l: its tile (binary search over s_pref) and rank
      int32_t id[kCcPer], l0[kCcPer], l1[kCcPer];
      uint32_t end[kCcPer];
#pragma unroll
      for (int k = 0; k < kCcPer; ++k) {
        const int l = tid + k * kCcBlock;
        id[k] = -1;
        l0[k] = l1[k] = -1;
        end[k] = 0;
        if (l < L) {
          int lo = 0, hi = nt - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pref[mid] <= l) lo = mid;
            else hi = mid - 1;
          }
          const int4 e = list[lo * kMaskTile + (l - s_pref[lo])];
          id[k] = e.x;
          end[k] = (((e.w >> 1) & 1) + ((e.w >> 2) & 1)) == 1 ? 1u : 0u;
          // each kept entry is hooked once, by its larger endpoint
          if (e.y >= 0 && e.y < e.x) {
            const int32_t p = map[e.y];
            l0[k] = s_pref[p / kMaskTile] + p % kMaskTile;
          }
          if (e.z >= 0 && e.z < e.x) {
            const int32_t p = map[e.z];
            l1[k] = s_pref[p / kMaskTile] + p % kMaskTile;
          }
          s_par[l] = l;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kCcPer; ++k) {
        const int l = tid + k * kCcBlock;
        if (l0[k] >= 0) lds_union(s_par, l, l0[k]);
        if (l1[k] >= 0) lds_union(s_par, l, l1[k]);
      }
      __syncthreads();
      int32_t r[kCcPer];
#pragma unroll
      for (int k = 0; k < kCcPer; ++k) {
        const int l = tid + k * kCcBlock;
        r[k] = l < L ? lds_find(s_par, l) : -1;
      }
      __syncthreads();
      // roots publish their ids, members take them as labels
#pragma unroll
      for (int k = 0; k < kCcPer; ++k)
        if (id[k] >= 0 && r[k] == tid + k * kCcBlock) s_par[r[k]] = id[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kCcPer; ++k)
        if (id[k] >= 0) J.label[id[k]] = s_par[r[k]];
      __syncthreads();
      // s_par becomes the per-root counter: 4 per read + 1 per path end
#pragma unroll
      for (int k = 0; k < kCcPer; ++k)
        if (id[k] >= 0) s_par[tid + k * kCcBlock] = 0;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kCcPer; ++k)
        if (id[k] >= 0) atomicAdd(s_par + r[k], 4 + (int)end[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kCcPer; ++k) {
        const int l = tid + k * kCcBlock;
        if (id[k] >= 0 && r[k] == l) J.parts.label_comp[id[k]] = s_par[l];
      }
      return;
    }
  }
  // too many reads for LDS: the job's own forest in global memory (only this
  // workgroup touches it), the list walked tile by tile
  const uint32_t tag = forest_tag(B);
  for (int t = 0; t < nt; ++t) {
    const int32_t c = cnt[t];
    for (int i = tid; i < c; i += kCcBlock) {
      const int4 e = list[t * kMaskTile + i];
      if (e.y >= 0 && e.y < e.x) tf_union(J.forest, tag, e.x, e.y);
      if (e.z >= 0 && e.z < e.x) tf_union(J.forest, tag, e.x, e.z);
    }
  }
  __syncthreads();
  for (int t = 0; t < nt; ++t) {
    const int32_t c = cnt[t];
    for (int i = tid; i < c; i += kCcBlock) {
      const int4 e = list[t * kMaskTile + i];
      int32_t r = e.x;
      while (true) {
        const int32_t p = tf_parent(J.forest, tag, r);
        if (p == r) break;
        r = p;
      }
      J.label[e.x] = r;
      const uint32_t degL = ((e.w >> 1) & 1) + ((e.w >> 2) & 1);
      atomicAdd((uint32_t *)J.parts.label_comp + r, 4u + (degL == 1 ? 1u : 0u));
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
  const BJob &J = B.jobs[B.tile_job[t]];
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
  const BJob &J = B.jobs[B.tile_job[t]];
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
    } else {
      J.parts.label_comp[v] = -1;
    }
  }
  if (t == J.vt_first + J.vt_count - 1 && threadIdx.x == 0) *J.parts.d_n_comp = base + tot;
}

// 4. LPT per job (one workgroup each), bin offsets, bucket cursors; the last
// workgroup lays out the batch-wide component and piece item ranges
constexpr int kBatchSortCap = 2048;
constexpr int kBatchBinCap = 256;

__global__ __launch_bounds__(kLptBlock) void kb_lpt(BatchDev B) {
  __shared__ uint64_t s_keys[kBatchSortCap];
  __shared__ int32_t s_bin[kBatchSortCap];
  __shared__ uint64_t s_binA[kBatchBinCap], s_binB[kBatchBinCap];
  __shared__ int64_t sh[kLptBlock / kWave + 1];
  const int j = blockIdx.x;
  const BJob &J = B.jobs[j];
  const int P = J.P;
  const int nc = *J.parts.d_n_comp;
  int m_e;
  if (nc <= kBatchSortCap && P <= kBatchBinCap)
    m_e = lpt_body(nc, P, J.parts.comp_size, s_keys, s_bin, s_binA, s_binB, J.parts.comp_bin,
                   J.parts.comp_rank, J.parts.comp_start, J.parts.bin_load, J.parts.comp_kind,
                   J.s.estart);
  else
    m_e = lpt_body(nc, P, J.parts.comp_size, J.s.keys, J.s.aux, J.s.bins, J.s.bins + P,
                   J.parts.comp_bin, J.parts.comp_rank, J.parts.comp_start, J.parts.bin_load,
                   J.parts.comp_kind, J.s.estart);
  __syncthreads();
  // branch vertices and kept entries of the job (BranchRemoval's counts)
  {
    int64_t nb = 0, ml = 0;
    for (int64_t v = threadIdx.x; v < J.g.n; v += kLptBlock) {
      const uint32_t f = J.flags[v];
      nb += f & 1;
      ml += ((f >> 1) & 1) + ((f >> 2) & 1);
    }
    int64_t tnb, tml;
    (void)block_excl_scan<int64_t, kLptBlock>(nb, sh, &tnb);
    (void)block_excl_scan<int64_t, kLptBlock>(ml, sh, &tml);
    if (threadIdx.x == 0) {
      J.counts[0] = (int32_t)tnb;
      J.counts[1] = (int32_t)tml;
    }
  }
  int64_t carry = 0;
  for (int base = 0; base < P; base += kLptBlock) {
    const int b = base + threadIdx.x;
    const int64_t x = b < P ? (int64_t)J.parts.bin_load[b] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, kLptBlock>(x, sh, &tot);
    if (b < P) J.local.bin_vptr[b] = (int32_t)(carry + ex);
    carry += tot;
  }
  for (int c = threadIdx.x; c < nc; c += kLptBlock) J.s.fill[c] = 0;
  __shared__ int last;
  if (threadIdx.x == 0) {
    J.local.bin_vptr[P] = (int32_t)carry;
    J.local.d_sizes[0] = (int32_t)carry;
    J.local.d_sizes[1] = m_e;
    J.local.loc_row_ptr[carry] = m_e;
    __threadfence();
    last = atomicAdd(&B.counters[2], 1u) == (unsigned)B.n_jobs - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  int64_t cc = 0, pc = 0, hc = 0;
  for (int base = 0; base < B.n_jobs; base += kLptBlock) {
    const int i = base + threadIdx.x;
    int64_t xc = 0, xp = 0;
    if (i < B.n_jobs) {
      const BJob &K = B.jobs[i];
      xc = __hip_atomic_load(K.parts.d_n_comp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      xp = __hip_atomic_load(K.local.bin_vptr + K.P, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int64_t xh = (xp + kWave - 1) / kWave;
    int64_t tc, tp, th;
    const int64_t ec = block_excl_scan<int64_t, kLptBlock>(xc, sh, &tc);
    const int64_t ep = block_excl_scan<int64_t, kLptBlock>(xp, sh, &tp);
    const int64_t eh = block_excl_scan<int64_t, kLptBlock>(xh, sh, &th);
    if (i < B.n_jobs) {
      B.comp_base[i] = (int32_t)(cc + ec);
      B.piece_base[i] = (int32_t)(pc + ep);
      B.chunk_base[i] = (int32_t)(hc + eh);
    }
    cc += tc;
    pc += tp;
    hc += th;
  }
  if (threadIdx.x == 0) {
    B.comp_base[B.n_jobs] = (int32_t)cc;
    B.piece_base[B.n_jobs] = (int32_t)pc;
    B.chunk_base[B.n_jobs] = (int32_t)hc;
    B.counters[2] = 0;
    B.counters[3] += 1u;  // the next run's forest tag
    __threadfence();
  }
}

// 5. each eligible read claims a slot in its component's block
template <int T>
__global__ __launch_bounds__(T) void kb_fill(BatchDev B) {
  const int t = blockIdx.x;
  const BJob &J = B.jobs[B.tile_job[t]];
  const int64_t v = (int64_t)(t - J.vt_first) * T + threadIdx.x;
  if (v >= J.g.n) return;
  const int32_t c = J.parts.label_comp[J.label[v]];
  if (c < 0) return;
  const uint32_t slot = atomicAdd(J.s.fill + c, 1u);
  J.s.tmp[J.parts.comp_start[c] + slot] = (int32_t)v;
}

// 6. induced subgraph of each component: sorted local numbers and local CSR
// rows (persistent over all components of the batch)
__global__ __launch_bounds__(kIndBlock) void kb_induce(BatchDev B) {
  __shared__ int32_t a[kIndLocalCap];
  __shared__ int32_t sh_scan[kIndBlock / kWave + 1];
  const int32_t total = B.comp_base[B.n_jobs];
  for (int32_t i = blockIdx.x; i < total; i += gridDim.x) {
    const int j = job_of(B.comp_base, B.n_jobs, i);
    const BJob &J = B.jobs[j];
    const int c = i - B.comp_base[j];
    induce_component(J.parts.comp_size[c], J.parts.comp_start[c], J.s.estart[c], J.s.tmp, J.flags,
                     J.g.row_ptr, J.g.col, J.local.perm, J.s.lidx, J.local.loc_row_ptr,
                     J.local.loc_col, J.local.loc_eid, a, sh_scan);
  }
}

// 7. walk every component (persistent, all components)
__global__ __launch_bounds__(kWalkBlock) void kb_walk(BatchDev B) {
  __shared__ int32_t s_nb[2 * kWalkCap], s_eid[2 * kWalkCap], s_nxt[2 * kWalkCap],
      s_dist[2 * kWalkCap], s_endv[2 * kWalkCap];
  __shared__ uint32_t sh_scan[kWalkBlock / kWave + 1];
  const int32_t total = B.comp_base[B.n_jobs];
  for (int32_t i = blockIdx.x; i < total; i += gridDim.x) {
    const int j = job_of(B.comp_base, B.n_jobs, i);
    const BJob &J = B.jobs[j];
    const int c = i - B.comp_base[j];
    const int q = J.parts.comp_size[c];
    const int st = J.parts.comp_start[c];
    if (q <= kWalkCap) {
      WalkArrays w{s_nb, s_eid, s_nxt, s_dist, s_endv};
      walk_component<true>(c, q, st, w, J.g, J.parts, J.local.perm, J.local.loc_row_ptr,
                           J.local.loc_col, J.local.loc_eid, J.out, J.s, nullptr, sh_scan);
    } else {
      const int64_t n = J.g.n;
      int32_t *gb = J.s.walk;
      WalkArrays w{gb + 2 * (int64_t)st, gb + 2 * n + 2 * (int64_t)st, gb + 4 * n + 4 * (int64_t)st,
                   gb + 8 * n + 4 * (int64_t)st, gb + 12 * n + 4 * (int64_t)st};
      walk_component<false>(c, q, st, w, J.g, J.parts, J.local.perm, J.local.loc_row_ptr,
                            J.local.loc_col, J.local.loc_eid, J.out, J.s, nullptr, sh_scan);
    }
  }
}

// 8. contig word offsets per job
__global__ __launch_bounds__(kScanBlock) void kb_offsets(BatchDev B) {
  __shared__ unsigned long long sh[kScanBlock / kWave + 1];
  const BJob &J = B.jobs[blockIdx.x];
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

// 9. packed copy: waves take chunks of 64 consecutive pieces of the batch
__device__ __forceinline__ PieceArrays piece_arrays(const BJob &J) {
  return piece_arrays(J.s.lay_contig, J.out.layout_vid, J.out.layout_rev, J.s.piece_off,
                      J.s.piece_len, J.g.read_off, J.g.read_len, J.out.len, J.out.base_off);
}

__global__ void kb_copy(BatchDev B) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t gw = blockIdx.x * (blockDim.x / kWave) + wave;
  const int32_t nwv = gridDim.x * (blockDim.x / kWave);
  const int32_t total = B.chunk_base[B.n_jobs];
  for (int32_t ch = gw; ch < total; ch += nwv) {
    // a chunk never spans two jobs, so the job is the same for the whole wave
    const int j = job_of(B.chunk_base, B.n_jobs, ch);
    const BJob &J = B.jobs[j];
    if (*J.out.d_total_words > J.out.cap_words) continue;
    const int32_t n_e = B.piece_base[j + 1] - B.piece_base[j];
    const int32_t c0 = (ch - B.chunk_base[j]) * kWave;
    const int cnt = n_e - c0 < kWave ? n_e - c0 : kWave;
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
      (g.n > 0 && (!g.read_len || !g.read_off || !g.seq)))
    return set_error(CG_EINVAL, "job %d: bad graph", i);
  if (J.P < 1 || J.P > 65536) return set_error(CG_EINVAL, "job %d: P=%d outside [1, 65536]", i, J.P);
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
  const size_t o_counters = take(sizeof(unsigned int) * 8);
  const size_t o_order = take(sizeof(int32_t) * n_jobs);
  int32_t n_mt = 0;
  for (int i = 0; i < n_jobs; ++i) {
    hj[i].mt_first = n_mt;
    hj[i].mt_count = (jobs[i].g.n + kMaskTile - 1) / kMaskTile;
    n_mt += hj[i].mt_count;
  }
  const size_t o_mtiles = take(sizeof(MaskTile) * (n_mt > 0 ? n_mt : 1));
  const size_t o_mtconn = take(sizeof(int32_t) * (n_mt > 0 ? n_mt : 1));
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
  b->prm = prm;
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
    }
    std::vector<MaskTile> mt;
    mt.reserve(n_mt);
    int32_t *d_mtconn = (int32_t *)(b->mem + o_mtconn);
    for (int i = 0; i < n_jobs; ++i)
      for (int32_t v0 = 0; v0 < jobs[i].g.n; v0 += kMaskTile)
        mt.push_back(MaskTile{jobs[i].g.row_ptr, jobs[i].g.col, jobs[i].flags, jobs[i].label,
                              jobs[i].parts.label_comp, hj[i].conn_list, hj[i].conn_map,
                              d_mtconn + (int32_t)mt.size(), jobs[i].g.n, v0});
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
  d.counters = (unsigned int *)(b->mem + o_counters);
  d.mt_conn = (int32_t *)(b->mem + o_mtconn);
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
  if (B.n_mtiles > 0)
    CG_LAUNCH(ctx, kb_mask_list, dim3(B.n_mtiles), dim3(kMaskThreads), st, B.mtiles);
  CG_LAUNCH(ctx, kb_cc_local, dim3(b->n_jobs), dim3(kCcBlock), st, B);
  if (T == 256) launch_vertex_phases<256>(b, st);
  else if (T == 512) launch_vertex_phases<512>(b, st);
  else launch_vertex_phases<1024>(b, st);
  CG_LAUNCH(ctx, kb_lpt, dim3(b->n_jobs), dim3(kLptBlock), st, B);
  if (T == 256) launch_vertex_fill<256>(b, st);
  else if (T == 512) launch_vertex_fill<512>(b, st);
  else launch_vertex_fill<1024>(b, st);
  CG_LAUNCH(ctx, kb_induce, dim3(PB), dim3(kIndBlock), st, B);
  CG_LAUNCH(ctx, kb_walk, dim3(PB), dim3(kWalkBlock), st, B);
  CG_LAUNCH(ctx, kb_offsets, dim3(b->n_jobs), dim3(kScanBlock), st, B);
  CG_LAUNCH(ctx, kb_copy, dim3(PB), dim3(b->prm.copy_block), st, B);
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
