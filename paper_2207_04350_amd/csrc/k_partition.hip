// Contig sizes and GreedyPartitioning (Sections 4.2 and 4.3).
//
//  k_part_zero / k_part_count  per-label counter (4 per read, +1 per read of
//                              degree 1 in L): size q = c >> 2, roots of degree
//                              one = c & 3 (2 for a path, 0 for a cycle)
//  k_part_compact              eligible components in ascending label order
//                              (single-pass look-back scan), label -> index map
//  k_part_wzero / k_part_weight bases weights (lengths of a component's reads)
//  k_part_lpt                  one workgroup: sort by (weight desc, label asc),
//                              exact LPT, sort by (bin, label), read offsets
#include "cg_device.h"

namespace cg {

constexpr int kPartBlock = 256;

__global__ __launch_bounds__(kPartBlock) void k_part_zero(int32_t n, int32_t *__restrict__ cnt) {
  const int64_t v = (int64_t)blockIdx.x * kPartBlock + threadIdx.x;
  if (v < n) cnt[v] = 0;
}

__global__ __launch_bounds__(kPartBlock) void k_part_count(int32_t n, const uint8_t *__restrict__ flags,
                                                           const int32_t *__restrict__ label,
                                                           int32_t *cnt) {
  const int64_t v = (int64_t)blockIdx.x * kPartBlock + threadIdx.x;
  if (v >= n) return;
  const uint32_t f = flags[v];
  const uint32_t degL = ((f >> 1) & 1) + ((f >> 2) & 1);
  atomicAdd((uint32_t *)cnt + label[v], 4u + (degL == 1 ? 1u : 0u));
}

// kCompactPer consecutive reads per thread, so that every block of a large
// graph is resident at once and the look-back chain is short
constexpr int kCompactPer = 4;
__global__ __launch_bounds__(kScanBlock) void k_part_compact(
    int32_t n, const uint8_t *__restrict__ flags, int32_t *label_comp, int32_t min_reads,
    int32_t *__restrict__ comp_label, int32_t *__restrict__ comp_size,
    uint8_t *__restrict__ comp_kind, int32_t *__restrict__ d_n_comp, ScanCtx sc, int nblocks) {
  const int blk = lookback_ticket(sc);
  const int64_t v0 = ((int64_t)blk * kScanBlock + threadIdx.x) * kCompactPer;
  uint32_t c[kCompactPer];
  bool elig[kCompactPer];
  uint32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < kCompactPer; ++k) {
    const int64_t v = v0 + k;
    c[k] = v < n ? (uint32_t)label_comp[v] : 0u;
    elig[k] = v < n && (c[k] >> 2) >= (uint32_t)min_reads && !(flags[v] & 1);
    cnt += elig[k] ? 1u : 0u;
  }
  unsigned long long incl_end;
  unsigned long long ex = lookback_block_scan(sc, blk, (unsigned long long)cnt, &incl_end);
#pragma unroll
  for (int k = 0; k < kCompactPer; ++k) {
    const int64_t v = v0 + k;
    if (v >= n) continue;
    if (elig[k]) {
      const uint32_t q = c[k] >> 2;
      comp_label[ex] = (int32_t)v;
      comp_size[ex] = (int32_t)q;
      comp_kind[ex] = q == 1 ? CG_KIND_SINGLE : ((c[k] & 3u) ? CG_KIND_PATH : CG_KIND_CYCLE);
      label_comp[v] = (int32_t)ex;
      ++ex;
    } else {
      label_comp[v] = -1;
    }
  }
  if (blk == nblocks - 1 && threadIdx.x == 0) *d_n_comp = (int32_t)incl_end;
  lookback_finish(sc, nblocks);
}

// ---------------------------------------------------------------------------
// Single-workgroup sort + LPT.
// ---------------------------------------------------------------------------
// bases weight of each eligible component: the lengths of its reads
__global__ __launch_bounds__(kPartBlock) void k_part_wzero(int32_t n, uint64_t *__restrict__ w) {
  const int64_t v = (int64_t)blockIdx.x * kPartBlock + threadIdx.x;
  if (v < n) w[v] = 0;
}

__global__ __launch_bounds__(kPartBlock) void k_part_weight(int32_t n, const int32_t *__restrict__ label,
                                                            const int32_t *__restrict__ label_comp,
                                                            const uint32_t *__restrict__ read_len,
                                                            uint64_t *w) {
  const int64_t v = (int64_t)blockIdx.x * kPartBlock + threadIdx.x;
  if (v >= n) return;
  const int32_t c = label_comp[label[v]];
  if (c >= 0) atomicAdd((unsigned long long *)w + c, (unsigned long long)read_len[v]);
}

__global__ __launch_bounds__(kLptBlock) void k_part_lpt(int32_t P, const int32_t *__restrict__ d_n_comp,
                                                        const int32_t *__restrict__ comp_size,
                                                        const uint64_t *__restrict__ weight,
                                                        uint64_t *bin_reads, unsigned int *status,
                                                        int32_t *__restrict__ comp_bin,
                                                        int32_t *__restrict__ comp_rank,
                                                        int32_t *__restrict__ comp_start,
                                                        uint64_t *__restrict__ bin_load,
                                                        uint64_t *g_keys, int32_t *g_bin,
                                                        uint64_t *g_bins) {
  __shared__ uint64_t s_keys[kSortCapLds];
  __shared__ int32_t s_bin[kSortCapLds];
  __shared__ uint64_t s_binA[kBinCapLds], s_binB[kBinCapLds];
  const int nc = *d_n_comp;
  if (nc <= kSortCapLds && P <= kBinCapLds)
    lpt_body<kLptBlock>(nc, P, comp_size, weight, s_keys, s_bin, s_binA, s_binB, comp_bin, comp_rank,
             comp_start, bin_load, bin_reads, status);
  else
    lpt_body<kLptBlock>(nc, P, comp_size, weight, g_keys, g_bin, g_bins, g_bins + P, comp_bin, comp_rank,
             comp_start, bin_load, bin_reads, status);
}

int launch_partition(cg_ctx *ctx, const cg_graph &g, const Scratch &s, const uint8_t *flags,
                     const int32_t *label, int32_t P, int32_t min_reads, int32_t weight,
                     const cg_parts &out, hipStream_t st) {
  const PhaseRange range("cg: GreedyPartitioning");
  const int32_t n = g.n;
  if (min_reads < 1) min_reads = 1;
  const int grid = n > 0 ? (int)((n + kPartBlock - 1) / kPartBlock) : 1;
  if (n > 0) {
    CG_LAUNCH(ctx, k_part_zero, dim3(grid), dim3(kPartBlock), st, n, out.label_comp);
    CG_LAUNCH(ctx, k_part_count, dim3(grid), dim3(kPartBlock), st, n, flags, label,
                       out.label_comp);
  }
  const int nb = scan_blocks(n > 0 ? (n + kCompactPer - 1) / kCompactPer : 1);
  CG_LAUNCH(ctx, k_part_compact, dim3(nb), dim3(kScanBlock), st, n, flags, out.label_comp,
                     min_reads, out.comp_label, out.comp_size, out.comp_kind, out.d_n_comp,
                     scan_ctx(ctx, s), nb);
  const bool bases = weight == CG_WEIGHT_BASES;
  if (bases && n > 0) {
    CG_LAUNCH(ctx, k_part_wzero, dim3(grid), dim3(kPartBlock), st, n, s.comp_w);
    CG_LAUNCH(ctx, k_part_weight, dim3(grid), dim3(kPartBlock), st, n, label, out.label_comp,
                       g.read_len, s.comp_w);
  }
  CG_LAUNCH(ctx, k_part_lpt, dim3(1), dim3(kLptBlock), st, P, out.d_n_comp, out.comp_size,
                     bases ? (const uint64_t *)s.comp_w : nullptr, s.bin_reads,
                     &ctx->fixed->status, out.comp_bin, out.comp_rank, out.comp_start,
                     out.bin_load, s.keys, s.aux, s.bins);
  return hip_check(hipGetLastError(), "k_part");
}

}  // namespace cg
