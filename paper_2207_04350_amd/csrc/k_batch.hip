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
// Every counter a launch uses is reset by the launch itself, so the eleven
// launches can be captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

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
  int32_t vt_first, vt_count;  // the job's vertex tiles (covering 0..n)
};

struct BatchDev {
  BJob *jobs;                       // [n_jobs]
  int32_t *tile_job;                // [n_vtiles]
  int32_t *tile_cnt;                // [n_vtiles] eligible roots per tile
  int32_t *comp_base;               // [n_jobs + 1] first component item of each job
  int32_t *piece_base;              // [n_jobs + 1] first piece item of each job
  int32_t *chunk_base;              // [n_jobs + 1] first 64-piece copy chunk of each job
  unsigned int *counters;           // [8] 2: LPT ticket
  Fixed *fixed;
  int32_t n_jobs, n_vtiles;
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
// 1. mask + label init + size-counter reset (one thread per vertex); the
// branch / kept-entry counts are summed later by the job's LPT workgroup
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(T) void kb_mask(BatchDev B) {
  const int t = blockIdx.x;
  const int j = B.tile_job[t];
  const BJob &J = B.jobs[j];
  const int32_t n = J.g.n;
  const int64_t v = (int64_t)(t - J.vt_first) * T + threadIdx.x;
  const bool live = v < n;
  const int32_t *row_ptr = J.g.row_ptr;
  int32_t b = v <= n ? row_ptr[v] : 0;
  int32_t nxt = __shfl_down(b, 1);
  if (lane_id() == kWave - 1 && live) nxt = row_ptr[v + 1];
  if (live) {
    J.flags[v] = (uint8_t)vertex_flags(row_ptr, J.g.col, b, nxt - b);
    J.label[v] = (int32_t)v;
    J.parts.label_comp[v] = 0;
  }
}

// 2. union-find hooks
template <int T>
__global__ __launch_bounds__(T) void kb_hook(BatchDev B) {
  const int t = blockIdx.x;
  const BJob &J = B.jobs[B.tile_job[t]];
  const int64_t v = (int64_t)(t - J.vt_first) * T + threadIdx.x;
  if (v >= J.g.n) return;
  const uint32_t f = J.flags[v];
  if (!(f & 6)) return;
  const int32_t b = J.g.row_ptr[v];
  if (f & 2) {
    const int32_t u = J.g.col[b];
    if (u > v) uf_union(J.label, (int32_t)v, u);
  }
  if (f & 4) {
    const int32_t u = J.g.col[b + 1];
    if (u > v) uf_union(J.label, (int32_t)v, u);
  }
}

// 3. compression to the root (= smallest id) and component size counters:
// a vertex's own root is final once all hooks are done, so it can count
// itself without waiting for the other vertices
template <int T>
__global__ __launch_bounds__(T) void kb_compress_count(BatchDev B) {
  const int t = blockIdx.x;
  const BJob &J = B.jobs[B.tile_job[t]];
  const int64_t v = (int64_t)(t - J.vt_first) * T + threadIdx.x;
  if (v >= J.g.n) return;
  int32_t *label = J.label;
  int32_t p = ld_relaxed(label + v);
  if (p != (int32_t)v) {
    while (true) {
      const int32_t q = ld_relaxed(label + p);
      if (q == p) break;
      p = q;
    }
    st_relaxed(label + v, p);
  }
  const uint32_t f = J.flags[v];
  const uint32_t degL = ((f >> 1) & 1) + ((f >> 2) & 1);
  atomicAdd((uint32_t *)J.parts.label_comp + p, 4u + (degL == 1 ? 1u : 0u));
}

// 4. eligible components in label order, reduce-then-scan: each tile counts
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

// 5. LPT per job (one workgroup each), bin offsets, bucket cursors; the last
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
    __threadfence();
  }
}

// 6. each eligible read claims a slot in its component's block
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

// 7. induced subgraph of each component: sorted local numbers and local CSR
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

// 8. walk every component (persistent, all components)
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

// 9. contig word offsets per job
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

// 10. packed copy: waves take chunks of 64 consecutive pieces of the batch
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
  return CG_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <int T>
static void launch_vertex_phases(cg_batch *b, hipStream_t st) {
  cg_ctx *ctx = b->ctx;
  const BatchDev &B = b->dev;
  CG_LAUNCH(ctx, kb_mask<T>, dim3(b->n_vtiles), dim3(T), st, B);
  CG_LAUNCH(ctx, kb_hook<T>, dim3(b->n_vtiles), dim3(T), st, B);
  CG_LAUNCH(ctx, kb_compress_count<T>, dim3(b->n_vtiles), dim3(T), st, B);
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
  for (int i = 0; i < n_jobs; ++i)
    job_off[i] = take(layout(jobs[i].g.n, jobs[i].g.m, jobs[i].P).total);
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
    }
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
