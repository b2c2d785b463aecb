// The step before the path (Algorithm 1: Prune(IsContainedRead), then
// TransitiveReduction; Section 2 defines redundant vertices and redundant
// edges) on an overlap graph R given like a string graph:
//
//  k_red_contained  one thread per read: a read is contained when an entry
//                   covers all of it (ovl >= len) from a longer read, or an
//                   equally long one with a smaller id
//  k_red_trans      one wave per row u, the row in LDS up to kRedCap entries:
//                   for every neighbour v of u the lanes walk v's row and
//                   look its columns x up in u's row; entry u->x is marked
//                   transitive when u, v, x is a valid walk with u->x's end
//                   orientations and overhangs that add up to u->x's
//  k_red_keep       one wave per row: an entry stays when neither read is
//                   contained and neither it nor its twin is marked; entries
//                   kept per row
//  k_red_rows       row pointers of the string graph (look-back scan)
//  k_red_compact    one wave per row: the kept entries in R's column order
//
// kept[e] carries the mark in bit 0 (k_red_trans), the decision in bit 1
// (k_red_keep), and ends as 0 / 1 (k_red_compact).
#include "cg_device.h"

namespace cg {

constexpr int kRedBlock = 256;
constexpr int kRedCap = 1024;  // row entries held in LDS by k_red_trans

__global__ __launch_bounds__(kRedBlock) void k_red_contained(cg_graph g, uint8_t *contained) {
  const int64_t v = (int64_t)blockIdx.x * kRedBlock + threadIdx.x;
  if (v >= g.n) return;
  const uint32_t lv = g.read_len[v];
  uint8_t c = 0;
  for (int32_t e = g.row_ptr[v]; e < g.row_ptr[v + 1]; ++e) {
    const int32_t u = g.col[e];
    const uint32_t lu = g.read_len[u];
    if (g.ovl[e] >= lv && (lu > lv || (lu == lv && u < v))) c = 1;
  }
  contained[v] = c;
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

__global__ __launch_bounds__(kWave) void k_red_trans(cg_graph g, uint32_t fuzz,
                                                      const uint8_t *__restrict__ contained,
                                                      uint8_t *kept) {
  __shared__ int32_t s_col[kRedCap];
  __shared__ uint32_t s_ovl[kRedCap];
  __shared__ uint8_t s_str[kRedCap], s_mark[kRedCap];
  const int32_t u = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t a = g.row_ptr[u], du = g.row_ptr[u + 1] - a;
  if (contained[u]) {
    for (int i = lane; i < du; i += kWave) kept[a + i] = 0;
    return;
  }
  // u's row: in LDS, or read in place (marks then go straight to kept)
  const bool in_lds = du <= kRedCap;
  const int32_t *rc = g.col + a;
  const uint32_t *ro = g.ovl + a;
  const uint8_t *rs = g.strand + a;
  if (in_lds) {
    for (int i = lane; i < du; i += kWave) {
      s_col[i] = g.col[a + i];
      s_ovl[i] = g.ovl[a + i];
      s_str[i] = g.strand[a + i];
      s_mark[i] = 0;
    }
    rc = s_col;
    ro = s_ovl;
    rs = s_str;
  } else {
    for (int i = lane; i < du; i += kWave) kept[a + i] = 0;
    __threadfence_block();
  }
  __syncthreads();
  for (int32_t f = 0; f < du; ++f) {
    const int32_t v = rc[f];
    if (contained[v]) continue;
    const uint32_t suv = rs[f];
    const int64_t sfx_uv = (int64_t)g.read_len[v] - ro[f];
    const int32_t b = g.row_ptr[v], dv = g.row_ptr[v + 1] - b;
    for (int32_t i = lane; i < dv; i += kWave) {
      const int32_t x = g.col[b + i];
      if (x == u) continue;
      const int p = lower_bound_i32(rc, du, x);
      if (p == du || rc[p] != x) continue;
      const uint32_t svx = g.strand[b + i], sux = rs[p];
      // a valid walk u, v, x with u->x's end orientations
      if ((suv & 1u) != (sux & 1u) || ((suv >> 1) & 1u) != (svx & 1u) ||
          ((svx >> 1) & 1u) != ((sux >> 1) & 1u))
        continue;
      const int64_t lx = g.read_len[x];
      const int64_t sum = sfx_uv + (lx - (int64_t)g.ovl[b + i]);
      const int64_t sfx_ux = lx - (int64_t)ro[p];
      const int64_t diff = sum > sfx_ux ? sum - sfx_ux : sfx_ux - sum;
      if (diff <= (int64_t)fuzz) {
        if (in_lds) s_mark[p] = 1;
        else kept[a + p] = 1;
      }
    }
  }
  if (in_lds) {
    __syncthreads();
    for (int i = lane; i < du; i += kWave) kept[a + i] = s_mark[i];
  }
}

__global__ __launch_bounds__(kWave) void k_red_keep(cg_graph g,
                                                     const uint8_t *__restrict__ contained,
                                                     uint8_t *kept, int32_t *counts) {
  const int32_t u = blockIdx.x;
  const int lane = threadIdx.x;
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

__global__ __launch_bounds__(kWave) void k_red_compact(cg_graph g,
                                                        const int32_t *__restrict__ s_row_ptr,
                                                        uint8_t *kept, int32_t *__restrict__ s_col,
                                                        uint32_t *__restrict__ s_ovl,
                                                        uint8_t *__restrict__ s_strand) {
  const int32_t u = blockIdx.x;
  const int lane = threadIdx.x;
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
  const int32_t n = g.n;
  if (n > 0) {
    CG_LAUNCH(ctx, k_red_contained, dim3((n + kRedBlock - 1) / kRedBlock), dim3(kRedBlock), st,
              g, contained);
    CG_LAUNCH(ctx, k_red_trans, dim3(n), dim3(kWave), st, g, fuzz, contained, kept);
    CG_LAUNCH(ctx, k_red_keep, dim3(n), dim3(kWave), st, g, contained, kept, s.tmp);
  }
  const int nb = scan_blocks((int64_t)n + 1);
  CG_LAUNCH(ctx, k_red_rows, dim3(nb), dim3(kScanBlock), st, n, s.tmp, s_row_ptr, d_m,
            scan_ctx(ctx, s), nb);
  if (n > 0)
    CG_LAUNCH(ctx, k_red_compact, dim3(n), dim3(kWave), st, g, s_row_ptr, kept, s_col, s_ovl,
              s_strand);
  return hip_check(hipGetLastError(), "k_red");
}

}  // namespace cg
