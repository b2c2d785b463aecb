// The step before the path (Algorithm 1: Prune(IsContainedRead), then
// TransitiveReduction; Section 2 defines redundant vertices and redundant
// edges) on an overlap graph R given like a string graph.  Every row pass
// runs one wave per row, kRedRowWaves rows per workgroup:
//
//  k_red_contained  a read is contained when an entry covers all of it
//                   (ovl >= len) from a longer read, or an equally long one
//                   with a smaller id
//  k_red_trans      row u in LDS (up to kRedCap entries) with, for every
//                   neighbour v, where v's row starts, how many entries it
//                   has (none for a contained v) and v's length; the lanes
//                   then take the (v, v->x) pairs of all neighbours together
//                   and look each x up in u's row: entry u->x is marked
//                   transitive when u, v, x is a valid walk with u->x's end
//                   orientations and overhangs that add up to u->x's.  A
//                   longer row is read in place, one neighbour at a time.
//  k_red_keep       an entry stays when neither read is contained and
//                   neither it nor its twin is marked; entries kept per row
//  k_red_rows       row pointers of the string graph (look-back scan)
//  k_red_compact    the kept entries in R's column order
//
// kept[e] carries the mark in bit 0 (k_red_trans), the decision in bit 1
// (k_red_keep), and ends as 0 / 1 (k_red_compact).
//
// The overhang test: sfx(x->y) = len(y) - ovl(x->y), and
// sfx(u->v) + sfx(v->x) - sfx(u->x) = len(v) - ovl(u->v) - ovl(v->x) + ovl(u->x)
// (len(x) cancels), so x's length is never read.
#include "cg_device.h"

namespace cg {

constexpr int kRedRowWaves = 4;  // rows per workgroup of the row passes
constexpr int kRedRowBlock = kRedRowWaves * kWave;
constexpr int kRedCap = 256;     // row entries k_red_trans holds in LDS

// the row of the calling wave, or -1 past the last row (wave-uniform)
__device__ __forceinline__ int32_t red_row(int32_t n) {
  const int32_t u = (int32_t)blockIdx.x * kRedRowWaves +
                    __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  return u < n ? u : -1;
}

// LDS written by the lanes of a wave is seen by all of its lanes after this:
// a wave's LDS accesses are carried out in order, so this only keeps the
// compiler from moving accesses across it
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kRedRowBlock) void k_red_contained(cg_graph g, uint8_t *contained) {
  const int32_t v = red_row(g.n);
  if (v < 0) return;
  const int lane = lane_id();
  const int32_t a = g.row_ptr[v], d = g.row_ptr[v + 1] - a;
  const uint32_t lv = g.read_len[v];
  bool c = false;
  for (int32_t i = lane; i < d; i += kWave) {
    const int32_t u = g.col[a + i];
    const uint32_t lu = g.read_len[u];
    c = c || (g.ovl[a + i] >= lv && (lu > lv || (lu == lv && u < v)));
  }
  const bool any = __ballot(c) != 0ull;
  if (lane == 0) contained[v] = any ? 1 : 0;
}

// the first position in a[0, len) holding a value >= x
__device__ __forceinline__ int lower_bound_i32(const int32_t *a, int len, int32_t x) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// a valid walk u, v, x with u->x's end orientations (strand bits s = bit 0,
// d = bit 1 of u->v, v->x and u->x)
__device__ __forceinline__ bool same_ends(uint32_t suv, uint32_t svx, uint32_t sux) {
  return (suv & 1u) == (sux & 1u) && ((suv >> 1) & 1u) == (svx & 1u) &&
         ((svx >> 1) & 1u) == ((sux >> 1) & 1u);
}

__device__ __forceinline__ bool within(int64_t d, uint32_t fuzz) {
  return (d < 0 ? -d : d) <= (int64_t)fuzz;
}

// Row u longer than kRedCap, read in place: one neighbour at a time, marks
// straight to kept.
__device__ void red_trans_long(const cg_graph &g, uint32_t fuzz, const uint8_t *contained,
                               uint8_t *kept, int32_t u, int32_t a, int32_t du, int lane) {
  for (int i = lane; i < du; i += kWave) kept[a + i] = 0;
  __threadfence_block();  // the zeros land before any mark
  wave_lds_sync();
  const int32_t *rc = g.col + a;
  for (int32_t f = 0; f < du; ++f) {
    const int32_t v = rc[f];
    if (contained[v]) continue;
    const uint32_t suv = g.strand[a + f];
    const int64_t base = (int64_t)g.read_len[v] - g.ovl[a + f];
    const int32_t b = g.row_ptr[v], dv = g.row_ptr[v + 1] - b;
    for (int32_t i = lane; i < dv; i += kWave) {
      const int32_t x = g.col[b + i];
      if (x == u) continue;
      const int p = lower_bound_i32(rc, du, x);
      if (p == du || rc[p] != x) continue;
      if (!same_ends(suv, g.strand[b + i], g.strand[a + p])) continue;
      if (within(base - (int64_t)g.ovl[b + i] + (int64_t)g.ovl[a + p], fuzz)) kept[a + p] = 1;
    }
  }
}

__global__ __launch_bounds__(kRedRowBlock) void k_red_trans(cg_graph g, uint32_t fuzz,
                                                            const uint8_t *__restrict__ contained,
                                                            uint8_t *kept) {
  __shared__ int32_t sh_col[kRedRowWaves][kRedCap];
  __shared__ uint32_t sh_ovl[kRedRowWaves][kRedCap];
  __shared__ int32_t sh_vb[kRedRowWaves][kRedCap];       // first entry of neighbour f's row
  __shared__ int32_t sh_pfx[kRedRowWaves][kRedCap];  // pairs of the neighbours before f
  __shared__ uint32_t sh_vlen[kRedRowWaves][kRedCap];
  __shared__ uint8_t sh_str[kRedRowWaves][kRedCap], sh_mark[kRedRowWaves][kRedCap];
  const int32_t u = red_row(g.n);
  if (u < 0) return;
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  const int32_t a = g.row_ptr[u], du = g.row_ptr[u + 1] - a;
  if (contained[u]) {
    for (int i = lane; i < du; i += kWave) kept[a + i] = 0;
    return;
  }
  if (du > kRedCap) {
    red_trans_long(g, fuzz, contained, kept, u, a, du, lane);
    return;
  }
  int32_t *s_col = sh_col[w], *s_vb = sh_vb[w], *s_pfx = sh_pfx[w];
  uint32_t *s_ovl = sh_ovl[w], *s_vlen = sh_vlen[w];
  uint8_t *s_str = sh_str[w], *s_mark = sh_mark[w];
  // u's row and its neighbours' rows; the pair counts prefix-summed
  int32_t carry = 0;
  for (int32_t base = 0; base < du; base += kWave) {
    const int32_t i = base + lane;
    int32_t dv = 0;
    if (i < du) {
      const int32_t v = g.col[a + i];
      const int32_t b = g.row_ptr[v];
      s_col[i] = v;
      s_ovl[i] = g.ovl[a + i];
      s_str[i] = g.strand[a + i];
      s_mark[i] = 0;
      s_vb[i] = b;
      s_vlen[i] = g.read_len[v];
      dv = contained[v] ? 0 : g.row_ptr[v + 1] - b;
    }
    const int32_t inc = wave_incl_scan(dv);
    if (i < du) s_pfx[i] = carry + inc - dv;
    carry += __shfl(inc, kWave - 1);
  }
  wave_lds_sync();
  // pair t belongs to the last neighbour f with s_pfx[f] <= t (one with
  // entries: t < carry rules out an empty last neighbour)
  for (int32_t t = lane; t < carry; t += kWave) {
    int lo = 0, hi = du - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pfx[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int32_t e = s_vb[lo] + (t - s_pfx[lo]);
    const int32_t x = g.col[e];
    if (x == u) continue;
    const int p = lower_bound_i32(s_col, du, x);
    if (p == du || s_col[p] != x) continue;
    if (!same_ends(s_str[lo], g.strand[e], s_str[p])) continue;
    const int64_t d = (int64_t)s_vlen[lo] - (int64_t)s_ovl[lo] - (int64_t)g.ovl[e] + (int64_t)s_ovl[p];
    if (within(d, fuzz)) s_mark[p] = 1;
  }
  wave_lds_sync();
  for (int i = lane; i < du; i += kWave) kept[a + i] = s_mark[i];
}

__global__ __launch_bounds__(kRedRowBlock) void k_red_keep(cg_graph g,
                                                           const uint8_t *__restrict__ contained,
                                                           uint8_t *kept, int32_t *counts) {
  const int32_t u = red_row(g.n);
  if (u < 0) return;
  const int lane = lane_id();
  const int32_t a = g.row_ptr[u], du = g.row_ptr[u + 1] - a;
  const bool cu = contained[u] != 0;
  int32_t n_kept = 0;
  for (int i = lane; i < du; i += kWave) {
    const int32_t x = g.col[a + i];
    bool k = !cu && !contained[x] && !(kept[a + i] & 1u);
    if (k) {
      // the twin x->u: its mark decides as well
      const int32_t b = g.row_ptr[x], dx = g.row_ptr[x + 1] - b;
      const int q = lower_bound_i32(g.col + b, dx, u);
      if (q < dx && g.col[b + q] == u && (kept[b + q] & 1u)) k = false;
    }
    // bit 0 is left as it was: other rows read it as their twin's mark
    if (k) kept[a + i] = 2;
    n_kept += k ? 1 : 0;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) n_kept += __shfl_xor(n_kept, off);
  if (lane == 0) counts[u] = n_kept;
}

__global__ __launch_bounds__(kScanBlock) void k_red_rows(int32_t n, const int32_t *__restrict__ counts,
                                                         int32_t *__restrict__ s_row_ptr,
                                                         int32_t *__restrict__ d_m, ScanCtx sc,
                                                         int nblocks) {
  const int blk = lookback_ticket(sc);
  const int64_t i = (int64_t)blk * kScanBlock + threadIdx.x;
  const uint32_t c = i < n ? (uint32_t)counts[i] : 0u;
  unsigned long long incl_end;
  const unsigned long long ex = lookback_block_scan(sc, blk, c, &incl_end);
  if (i <= n) s_row_ptr[i] = (int32_t)ex;
  if (i == n) *d_m = (int32_t)ex;
  lookback_finish(sc, nblocks);
}

__global__ __launch_bounds__(kRedRowBlock) void k_red_compact(
    cg_graph g, const int32_t *__restrict__ s_row_ptr, uint8_t *kept, int32_t *__restrict__ s_col,
    uint32_t *__restrict__ s_ovl, uint8_t *__restrict__ s_strand) {
  const int32_t u = red_row(g.n);
  if (u < 0) return;
  const int lane = lane_id();
  const int32_t a = g.row_ptr[u], du = g.row_ptr[u + 1] - a;
  int32_t at = s_row_ptr[u];
  for (int32_t base = 0; base < du; base += kWave) {
    const int32_t i = base + lane;
    const bool k = i < du && (kept[a + i] & 2u);
    const uint64_t mask = __ballot(k);
    if (k) {
      const int32_t o = at + __popcll(mask & ((1ull << lane) - 1ull));
      s_col[o] = g.col[a + i];
      s_ovl[o] = g.ovl[a + i];
      s_strand[o] = g.strand[a + i];
    }
    if (i < du) kept[a + i] = k ? 1 : 0;
    at += __popcll(mask);
  }
}

int launch_reduce(cg_ctx *ctx, const cg_graph &g, const Scratch &s, uint32_t fuzz,
                  uint8_t *contained, uint8_t *kept, int32_t *s_row_ptr, int32_t *s_col,
                  uint32_t *s_ovl, uint8_t *s_strand, int32_t *d_m, hipStream_t st) {
  const PhaseRange range("cg: reduce");
  const int32_t n = g.n;
  const dim3 rows((n + kRedRowWaves - 1) / kRedRowWaves);
  if (n > 0) {
    CG_LAUNCH(ctx, k_red_contained, rows, dim3(kRedRowBlock), st, g, contained);
    CG_LAUNCH(ctx, k_red_trans, rows, dim3(kRedRowBlock), st, g, fuzz, contained, kept);
    CG_LAUNCH(ctx, k_red_keep, rows, dim3(kRedRowBlock), st, g, contained, kept, s.tmp);
  }
  const int nb = scan_blocks((int64_t)n + 1);
  CG_LAUNCH(ctx, k_red_rows, dim3(nb), dim3(kScanBlock), st, n, s.tmp, s_row_ptr, d_m,
            scan_ctx(ctx, s), nb);
  if (n > 0)
    CG_LAUNCH(ctx, k_red_compact, rows, dim3(kRedRowBlock), st, g, s_row_ptr, kept, s_col, s_ovl,
              s_strand);
  return hip_check(hipGetLastError(), "k_red");
}

}  // namespace cg
