// BranchRemoval (Section 4.2: degree = nonzeros of a row of S, branch vertex
// at degree >= 3, L = S without the rows and columns of branch vertices),
// ConnectedComponent (Section 4.2, labels = smallest vertex id of each
// component of L) and the input checks.
//
// Layout in HBM: CSR row_ptr/col of S, one flag byte per vertex (bit0 branch,
// bit1/bit2 entry 0/1 of the row kept), one int32 label per vertex.
#include "cg_device.h"

namespace cg {

// ---------------------------------------------------------------------------
// Mask: one thread per vertex, a grid of at most kMaskMaxBlocks workgroups
// striding over the vertices.  row_ptr[v+1] comes from the neighbouring lane
// (one coalesced load per lane); the at most two neighbours of a degree <= 2
// row are the only gathers.
// ---------------------------------------------------------------------------
constexpr int kMaskBlock = 512;

// Grids of at most this many workgroups add the counts up in the kernel
// (one release per workgroup); larger ones leave it to k_mask_sum.
constexpr int kMaskSumInKernel = 64;

__device__ __forceinline__ void store_counts(unsigned long long a, int32_t *d_counts) {
  d_counts[0] = (int32_t)(uint32_t)a;
  d_counts[1] = (int32_t)(uint32_t)(a >> 32);
}

__global__ __launch_bounds__(kMaskBlock) void k_mask(int32_t n, const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     uint8_t *__restrict__ flags, Fixed *fx,
                                                     int32_t *__restrict__ d_counts) {
  // counts: ballots per wave, summed per workgroup in LDS, one plain store
  // per workgroup of a packed word (branch reads low, kept entries high:
  // neither sum reaches 2^32).  A large grid leaves the sum to k_mask_sum
  // and uses no atomics and no fences (an agent-scope release writes the L2
  // back, which thousands of workgroups would each pay).
  __shared__ unsigned long long s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kMaskBlock;
  // every lane of a wave runs the same iterations (the bound is rounded up
  // to whole workgroups), so the shuffle and the ballots see the whole wave
  const int64_t end = ((int64_t)n + kMaskBlock - 1) / kMaskBlock * kMaskBlock;
  for (int64_t v = (int64_t)blockIdx.x * kMaskBlock + threadIdx.x; v < end; v += stride) {
    const bool live = v < n;
    const int32_t b = v <= n ? row_ptr[v] : 0;  // row_ptr has n+1 entries
    int32_t nxt = __shfl_down(b, 1);
    if (lane_id() == kWave - 1 && live) nxt = row_ptr[v + 1];
    const int32_t deg = live ? nxt - b : 0;
    uint32_t f = 0;
    if (live) {
      f = vertex_flags(row_ptr, col, b, deg);
      flags[v] = (uint8_t)f;
    }
    const uint32_t nb = (uint32_t)__popcll(__ballot(f & 1));
    const uint32_t ml = (uint32_t)(__popcll(__ballot(f & 2)) + __popcll(__ballot(f & 4)));
    if (lane_id() == 0 && (nb | ml)) atomicAdd(&s_cnt, (unsigned long long)ml << 32 | nb);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (gridDim.x == 1) {
    store_counts(s_cnt, d_counts);
    return;
  }
  fx->mask_part[blockIdx.x] = s_cnt;
  if (gridDim.x > kMaskSumInKernel) return;
  // the last workgroup out adds the parts up
  const unsigned t =
      __hip_atomic_fetch_add(&fx->mask_ticket, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  if (t != gridDim.x - 1) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  unsigned long long a = 0;
  for (unsigned i = 0; i < gridDim.x; ++i) a += fx->mask_part[i];
  store_counts(a, d_counts);
  fx->mask_ticket = 0;
}

// one workgroup: a few parts per thread (their loads issued together), then
// one block-wide sum (one wave looping over thousands of parts waited for a
// load per turn)
__global__ __launch_bounds__(kScanBlock) void k_mask_sum(int nparts, const Fixed *fx,
                                                         int32_t *__restrict__ d_counts) {
  __shared__ unsigned long long sh[kScanBlock / kWave + 1];
  unsigned long long a = 0;
  for (int i = threadIdx.x; i < nparts; i += kScanBlock) a += fx->mask_part[i];
  unsigned long long tot;
  (void)block_excl_scan<unsigned long long, kScanBlock>(a, sh, &tot);
  if (threadIdx.x == 0) store_counts(tot, d_counts);
}

int launch_mask(cg_ctx *ctx, const cg_graph &g, uint8_t *flags, int32_t *d_counts,
                hipStream_t st) {
  const PhaseRange range("cg: BranchRemoval");
  int64_t grid = ((int64_t)g.n + kMaskBlock - 1) / kMaskBlock;
  if (grid < 1) grid = 1;
  if (grid > kMaskMaxBlocks) grid = kMaskMaxBlocks;
  CG_LAUNCH(ctx, k_mask, dim3((unsigned)grid), dim3(kMaskBlock), st, g.n, g.row_ptr, g.col, flags,
            ctx->fixed, d_counts);
  if (grid > kMaskSumInKernel)
    CG_LAUNCH(ctx, k_mask_sum, dim3(1), dim3(kScanBlock), st, (int)grid, ctx->fixed, d_counts);
  return hip_check(hipGetLastError(), "k_mask");
}

// ---------------------------------------------------------------------------
// Components: union-find with min-id roots.  A root is always the smallest
// id of its tree (a larger root is only ever linked under a smaller one), so
// after full compression every vertex holds the smallest id of its
// component.  Links are made by compare-and-swap on the root, so concurrent
// hooks never lose a union; path halving only ever stores an ancestor.
// ---------------------------------------------------------------------------
constexpr int kCcBlock = 256;

__global__ __launch_bounds__(kCcBlock) void k_cc_init(int32_t n, int32_t *__restrict__ label) {
  const int64_t v = (int64_t)blockIdx.x * kCcBlock + threadIdx.x;
  if (v < n) label[v] = (int32_t)v;
}

__global__ __launch_bounds__(kCcBlock) void k_cc_hook(int32_t n, const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const uint8_t *__restrict__ flags,
                                                      int32_t *label) {
  const int64_t v = (int64_t)blockIdx.x * kCcBlock + threadIdx.x;
  if (v >= n) return;
  const uint32_t f = flags[v];
  if (!(f & 6)) return;
  const int32_t b = row_ptr[v];
  // each undirected kept edge is hooked once, from its smaller end
  if (f & 2) {
    int32_t u = col[b];
    if (u > v) uf_union(label, (int32_t)v, u);
  }
  if (f & 4) {
    int32_t u = col[b + 1];
    if (u > v) uf_union(label, (int32_t)v, u);
  }
}

__global__ __launch_bounds__(kCcBlock) void k_cc_compress(int32_t n, int32_t *label) {
  const int64_t v = (int64_t)blockIdx.x * kCcBlock + threadIdx.x;
  if (v >= n) return;
  int32_t x = (int32_t)v;
  int32_t p = ld_relaxed(label + x);
  if (p == x) return;
  while (true) {
    int32_t q = ld_relaxed(label + p);
    if (q == p) break;
    p = q;
  }
  st_relaxed(label + v, p);
}

int launch_components(cg_ctx *ctx, const cg_graph &g, const uint8_t *flags, int32_t *label,
                      hipStream_t st) {
  const PhaseRange range("cg: ConnectedComponent");
  (void)ctx;
  if (g.n == 0) return CG_OK;
  int grid = (int)((g.n + kCcBlock - 1) / kCcBlock);
  CG_LAUNCH(ctx, k_cc_init, dim3(grid), dim3(kCcBlock), st, g.n, label);
  CG_LAUNCH(ctx, k_cc_hook, dim3(grid), dim3(kCcBlock), st, g.n, g.row_ptr, g.col, flags,
                     label);
  CG_LAUNCH(ctx, k_cc_compress, dim3(grid), dim3(kCcBlock), st, g.n, label);
  return hip_check(hipGetLastError(), "k_cc");
}

// ---------------------------------------------------------------------------
// Validation.  Every failure is packed as (phase, index, reason) and the
// smallest packed value wins, which reproduces "first failure in check
// order".  Indices are clamped so that even a malformed row_ptr never sends a
// load outside the caller's arrays.
// ---------------------------------------------------------------------------
constexpr int kValBlock = 256;

__device__ __forceinline__ unsigned long long pack_fail(unsigned phase, int64_t idx, unsigned why) {
  return ((unsigned long long)phase << 60) | ((unsigned long long)idx << 4) | why;
}

__global__ void k_val_init(Fixed *fx) { fx->valid_best = ~0ull; }

__global__ __launch_bounds__(kValBlock) void k_val_check(cg_graph g, Fixed *fx) {
  const int64_t v = (int64_t)blockIdx.x * kValBlock + threadIdx.x;
  if (v == 0) {
    if (g.row_ptr[0] != 0 || g.row_ptr[g.n] != g.m) atomicMin(&fx->valid_best, pack_fail(0, 0, 1));
  }
  if (v >= g.n) return;
  const int32_t rb = g.row_ptr[v], re = g.row_ptr[v + 1];
  if (re < rb) atomicMin(&fx->valid_best, pack_fail(1, v, 1));
  {
    unsigned why = 0;
    uint32_t L = g.read_len[v];
    uint64_t off = g.read_off[v];
    if (L < 1) why = 9;
    else if (off % 16 != 0) why = 10;
    else if (off + L > g.seq_words * 16) why = 11;
    if (why) atomicMin(&fx->valid_best, pack_fail(2, v, why));
  }
  const int32_t lo = rb < 0 ? 0 : (rb > g.m ? g.m : rb);
  const int32_t hi = re < lo ? lo : (re > g.m ? g.m : re);
  for (int32_t j = lo; j < hi; ++j) {
    unsigned why = 0;
    int32_t u = g.col[j];
    if (u < 0 || u >= g.n) {
      why = 2;
    } else if (u == v) {
      why = 3;
    } else if (j > lo && g.col[j - 1] >= u) {
      why = 4;
    } else {
      int32_t tb = g.row_ptr[u], te = g.row_ptr[u + 1];
      tb = tb < 0 ? 0 : (tb > g.m ? g.m : tb);
      te = te < tb ? tb : (te > g.m ? g.m : te);
      int32_t t = -1;
      for (int32_t k = tb; k < te; ++k)
        if (g.col[k] == (int32_t)v) { t = k; break; }
      if (t < 0) {
        why = 5;
      } else if (g.ovl[t] != g.ovl[j]) {
        why = 6;
      } else {
        uint32_t sj = g.strand[j];
        uint32_t s = sj & 1, d = (sj >> 1) & 1;
        uint32_t want = (1 - d) | ((1 - s) << 1);
        if ((g.strand[t] & 3u) != want || (sj & ~3u)) {
          why = 7;
        } else {
          uint32_t lu = g.read_len[v], lv = g.read_len[u];
          uint32_t lmin = lu < lv ? lu : lv;
          if (g.ovl[j] < 1 || g.ovl[j] >= lmin) why = 8;
          else if (g.pre && g.pre[j] >= lu) why = 12;    // pre indexes the row's read
          else if (g.pre && g.post[j] >= lv) why = 13;   // post the column's read
        }
      }
    }
    if (why) {
      atomicMin(&fx->valid_best, pack_fail(3, j, why));
      break;
    }
  }
}

__global__ void k_val_final(Fixed *fx, int64_t *d_bad) {
  unsigned long long b = fx->valid_best;
  if (b == ~0ull) {
    d_bad[0] = -1;
    d_bad[1] = 0;
  } else {
    unsigned phase = (unsigned)(b >> 60);
    d_bad[0] = phase == 0 ? -2 : (int64_t)((b >> 4) & ((1ull << 56) - 1));
    d_bad[1] = (int64_t)(b & 15);
  }
}

int launch_validate(cg_ctx *ctx, const cg_graph &g, int64_t *d_bad, hipStream_t st) {
  const PhaseRange range("cg: validate");
  int grid = (int)((g.n + kValBlock - 1) / kValBlock);
  if (grid == 0) grid = 1;
  CG_LAUNCH(ctx, k_val_init, dim3(1), dim3(1), st, ctx->fixed);
  CG_LAUNCH(ctx, k_val_check, dim3(grid), dim3(kValBlock), st, g, ctx->fixed);
  CG_LAUNCH(ctx, k_val_final, dim3(1), dim3(1), st, ctx->fixed, d_bad);
  return hip_check(hipGetLastError(), "k_val");
}

}  // namespace cg
