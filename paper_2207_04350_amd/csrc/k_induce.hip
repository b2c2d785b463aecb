// InducedSubgraph (Section 4.3): V_i = reads owned by bin i, E_i = entries of
// L with both ends in V_i, renumbered locally with the global ids kept.  All
// bins share one local numbering ordered by (bin, label, id): a component's
// reads form the block [comp_start, comp_start + q).
//
//  k_ind_zero   bucket cursors; bin_vptr (scan of the reads of each bin); n_e
//  k_ind_fill   each eligible read claims a slot in its component's block
//  k_ind_local  one workgroup per component: sort the block by read id
//               (LDS bitonic up to 1024 reads, rank counting above)
//  k_ind_rows   local CSR rows (look-back scan of kept degrees), columns
//               renumbered through the local numbers, entry index kept;
//               k_ind_rows_wide does the same four rows per thread
#include "cg_device.h"

namespace cg {


constexpr int kIndBinLds = 2048;  // bins whose reads k_ind_zero sums in LDS
__global__ __launch_bounds__(kScanBlock) void k_ind_zero(int32_t P, const int32_t *__restrict__ d_n_comp,
                                                         const int32_t *__restrict__ comp_bin,
                                                         const int32_t *__restrict__ comp_size,
                                                         uint64_t *bin_reads,
                                                         uint32_t *__restrict__ fill,
                                                         int32_t *__restrict__ bin_vptr,
                                                         int32_t *__restrict__ d_sizes) {
  const int nc = *d_n_comp;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * blockDim.x)
    fill[c] = 0;
  if (blockIdx.x == 0) {
    // the reads of each bin (in LDS up to kIndBinLds bins, four components'
    // loads per thread issued together), then their prefix: bin_vptr
    __shared__ int64_t sh[kScanBlock / kWave + 1];
    __shared__ unsigned long long s_br[kIndBinLds];
    const bool lds = P <= kIndBinLds;
    if (lds) {
      for (int b = threadIdx.x; b < P; b += kScanBlock) s_br[b] = 0;
      __syncthreads();
      for (int c0 = threadIdx.x; c0 < nc; c0 += 4 * kScanBlock) {
        int32_t bb[4], sz[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = c0 + r * kScanBlock;
          bb[r] = c < nc ? comp_bin[c] : -1;
          sz[r] = c < nc ? comp_size[c] : 0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (bb[r] >= 0) atomicAdd(s_br + bb[r], (unsigned long long)sz[r]);
      }
    } else {
      for (int b = threadIdx.x; b < P; b += kScanBlock) bin_reads[b] = 0;
      __syncthreads();
      for (int c = threadIdx.x; c < nc; c += kScanBlock)
        atomicAdd((unsigned long long *)bin_reads + comp_bin[c], (unsigned long long)comp_size[c]);
    }
    __syncthreads();
    int64_t carry = 0;
    for (int base = 0; base < P; base += kScanBlock) {
      const int b = base + threadIdx.x;
      int64_t x = 0;
      if (b < P)
        x = lds ? (int64_t)s_br[b]
                : (int64_t)__hip_atomic_load(bin_reads + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int64_t tot;
      const int64_t ex = block_excl_scan<int64_t, kScanBlock>(x, sh, &tot);
      if (b < P) bin_vptr[b] = (int32_t)(carry + ex);
      carry += tot;
    }
    if (threadIdx.x == 0) {
      bin_vptr[P] = (int32_t)carry;
      d_sizes[0] = (int32_t)carry;
    }
  }
}

__global__ __launch_bounds__(kIndBlock) void k_ind_fill(int32_t n, const int32_t *__restrict__ label,
                                                        const int32_t *__restrict__ label_comp,
                                                        const int32_t *__restrict__ comp_start,
                                                        uint32_t *fill, int32_t *__restrict__ tmp) {
  const int64_t v = (int64_t)blockIdx.x * kIndBlock + threadIdx.x;
  if (v >= n) return;
  const int32_t c = label_comp[label[v]];
  if (c < 0) return;
  const uint32_t slot = atomicAdd(fill + c, 1u);
  tmp[comp_start[c] + slot] = (int32_t)v;
}

__global__ __launch_bounds__(kIndBlock) void k_ind_local(const int32_t *__restrict__ d_n_comp,
                                                         const int32_t *__restrict__ comp_size,
                                                         const int32_t *__restrict__ comp_start,
                                                         const int32_t *__restrict__ tmp,
                                                         int32_t *__restrict__ perm,
                                                         int32_t *__restrict__ lidx) {
  __shared__ int32_t a[kIndLocalCap];
  const int nc = *d_n_comp;
  for (int c = blockIdx.x; c < nc; c += gridDim.x)
    sort_component_block<kIndBlock, kIndLocalCap>(comp_size[c], comp_start[c], tmp + comp_start[c], perm, lidx, a);
}

__global__ __launch_bounds__(kScanBlock) void k_ind_rows(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const uint8_t *__restrict__ flags, const int32_t *__restrict__ bin_vptr, int32_t P,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ lidx,
    int32_t *__restrict__ loc_row_ptr, int32_t *__restrict__ loc_col,
    int32_t *__restrict__ loc_eid, int32_t *__restrict__ d_sizes, ScanCtx sc, int nblocks) {
  const int blk = lookback_ticket(sc);
  const int64_t i = (int64_t)blk * kScanBlock + threadIdx.x;
  const int32_t n_e = bin_vptr[P];
  // the grid covers every read and only the n_e reads of the contigs have
  // local numbers: blocks past them take no part in the scan (a block looks
  // back at lower tickets only, and the last block out clears every status)
  if ((int64_t)blk * kScanBlock > n_e) {
    lookback_finish(sc, nblocks);
    return;
  }
  int32_t v = -1;
  uint32_t f = 0;
  if (i < n_e) {
    v = perm[i];
    f = flags[v];
  }
  const uint32_t deg = ((f >> 1) & 1) + ((f >> 2) & 1);
  unsigned long long incl_end;
  const unsigned long long ex = lookback_block_scan(sc, blk, deg, &incl_end);
  if (i <= n_e) loc_row_ptr[i] = (int32_t)ex;
  if (i == n_e) d_sizes[1] = (int32_t)ex;
  if (i < n_e && deg) {
    const int32_t b = row_ptr[v];
    int32_t t = (int32_t)ex;
    if (f & 2) {
      loc_col[t] = lidx[col[b]];
      loc_eid[t] = b;
      ++t;
    }
    if (f & 4) {
      loc_col[t] = lidx[col[b + 1]];
      loc_eid[t] = b + 1;
    }
  }
  lookback_finish(sc, nblocks);
}

// k_ind_rows with kRowsWide consecutive local numbers per thread.  On a
// large graph it keeps four rows' loads in flight per thread and puts a
// quarter of the blocks in the look-back; on a small one, whose few thousand
// contig reads fill only a few dozen blocks, one row per thread spreads them
// over four times as many compute units and is the faster form.
constexpr int32_t kRowsWideReads = 1 << 19;  // reads from which the wide form runs
constexpr int kRowsWide = 4;
__global__ __launch_bounds__(kScanBlock) void k_ind_rows_wide(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const uint8_t *__restrict__ flags, const int32_t *__restrict__ bin_vptr, int32_t P,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ lidx,
    int32_t *__restrict__ loc_row_ptr, int32_t *__restrict__ loc_col,
    int32_t *__restrict__ loc_eid, int32_t *__restrict__ d_sizes, ScanCtx sc, int nblocks) {
  const int blk = lookback_ticket(sc);
  const int32_t n_e = bin_vptr[P];
  // the grid covers every read and only the n_e reads of the contigs have
  // local numbers: blocks past them take no part in the scan (a block looks
  // back at lower tickets only, and the last block out clears every status)
  if ((int64_t)blk * kScanBlock * kRowsWide > n_e) {
    lookback_finish(sc, nblocks);
    return;
  }
  const int64_t i0 = ((int64_t)blk * kScanBlock + threadIdx.x) * kRowsWide;
  // every load of the thread's rows is issued before the scan, level by
  // level (read, flags, row start, columns, their local numbers), and the
  // stores come after it: gfx9 counts loads and stores in one counter, so a
  // load behind a store would wait for it
  int32_t v[kRowsWide], b[kRowsWide], c0[kRowsWide], c1[kRowsWide];
  uint32_t f[kRowsWide];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kRowsWide; ++k) v[k] = i0 + k < n_e ? perm[i0 + k] : -1;
#pragma unroll
  for (int k = 0; k < kRowsWide; ++k) {
    f[k] = v[k] >= 0 ? flags[v[k]] : 0u;
    sum += ((f[k] >> 1) & 1) + ((f[k] >> 2) & 1);
  }
#pragma unroll
  for (int k = 0; k < kRowsWide; ++k) b[k] = (f[k] & 6u) ? row_ptr[v[k]] : 0;
#pragma unroll
  for (int k = 0; k < kRowsWide; ++k) {
    c0[k] = (f[k] & 2u) ? col[b[k]] : -1;
    c1[k] = (f[k] & 4u) ? col[b[k] + 1] : -1;
  }
#pragma unroll
  for (int k = 0; k < kRowsWide; ++k) {
    c0[k] = c0[k] >= 0 ? lidx[c0[k]] : -1;
    c1[k] = c1[k] >= 0 ? lidx[c1[k]] : -1;
  }
  unsigned long long incl_end;
  unsigned long long ex = lookback_block_scan(sc, blk, (unsigned long long)sum, &incl_end);
#pragma unroll
  for (int k = 0; k < kRowsWide; ++k) {
    const int64_t i = i0 + k;
    if (i <= n_e) loc_row_ptr[i] = (int32_t)ex;
    if (i == n_e) d_sizes[1] = (int32_t)ex;
    int32_t t = (int32_t)ex;
    if (f[k] & 2u) {
      loc_col[t] = c0[k];
      loc_eid[t] = b[k];
      ++t;
    }
    if (f[k] & 4u) {
      loc_col[t] = c1[k];
      loc_eid[t] = b[k] + 1;
      ++t;
    }
    ex = (unsigned long long)t;
  }
  lookback_finish(sc, nblocks);
}

int launch_induce(cg_ctx *ctx, const cg_graph &g, const Scratch &s, const uint8_t *flags,
                  const int32_t *label, const cg_parts &parts, int32_t P, const cg_local &out,
                  hipStream_t st) {
  const PhaseRange range("cg: InducedSubgraph");
  const int32_t n = g.n;
  const int zgrid = n > 0 ? (int)((n + kScanBlock - 1) / kScanBlock) : 1;
  CG_LAUNCH(ctx, k_ind_zero, dim3(zgrid < 256 ? zgrid : 256), dim3(kScanBlock), st, P,
                     parts.d_n_comp, parts.comp_bin, parts.comp_size, s.bin_reads, s.fill,
                     out.bin_vptr, out.d_sizes);
  if (n > 0) {
    const int grid = (int)((n + kIndBlock - 1) / kIndBlock);
    CG_LAUNCH(ctx, k_ind_fill, dim3(grid), dim3(kIndBlock), st, n, label, parts.label_comp,
                       parts.comp_start, s.fill, s.tmp);
    const int lgrid = n < 4096 ? n : 4096;
    CG_LAUNCH(ctx, k_ind_local, dim3(lgrid), dim3(kIndBlock), st, parts.d_n_comp,
                       parts.comp_size, parts.comp_start, s.tmp, out.perm, s.lidx);
  }
  if (n >= kRowsWideReads) {
    const int nb = scan_blocks(((int64_t)n + kRowsWide) / kRowsWide);
    CG_LAUNCH(ctx, k_ind_rows_wide, dim3(nb), dim3(kScanBlock), st, g.row_ptr, g.col, flags,
              out.bin_vptr, P, out.perm, s.lidx, out.loc_row_ptr, out.loc_col, out.loc_eid,
              out.d_sizes, scan_ctx(ctx, s), nb);
  } else {
    const int nb = scan_blocks((int64_t)n + 1);
    CG_LAUNCH(ctx, k_ind_rows, dim3(nb), dim3(kScanBlock), st, g.row_ptr, g.col, flags,
              out.bin_vptr, P, out.perm, s.lidx, out.loc_row_ptr, out.loc_col, out.loc_eid,
              out.d_sizes, scan_ctx(ctx, s), nb);
  }
  return hip_check(hipGetLastError(), "k_ind");
}

}  // namespace cg
